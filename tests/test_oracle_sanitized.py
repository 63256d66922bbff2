"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source is built a second time with -fsanitize=address,undefined
(every report fatal) and a child Python process runs it through the usual
ctypes wrapper over small cases that reach every part of it: frames with the
three smoothers (Sec. 4.5), one, two and six candidates (Sec. 4.3), lazy
refreshes between frames (Sec. 4.2), ARAP rows (Sec. 5.3, Eq. 8), flexible
beta, the hierarchy inspection calls, aggregation and colouring on their own.
The child must exit cleanly with no sanitizer report."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mgpbd_oracle.c")

CHILD = textwrap.dedent(r"""
    import numpy as np
    from oracle import oracle as O
    from paper_2505_13390_amd import workloads as W

    def frame(w, n_iters, frames=1, **kw):
        sim = O.Sim(w, O.default_opts(**kw))
        pos, vel = O.positions(w)
        for f in range(frames):
            sim.set_frame(f)
            r = sim.step(pos, vel, n_iters)
            assert r["status"] == 0, (kw, r["status"])
        return sim

    w = W.beam(8, 3, 3, seed=5, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9)
    for kw in ({}, {"smoother": 1}, {"smoother": 2}, {"n_cand": 2}, {"n_cand": 6},
               {"flexible": 1}, {"reuse_interval": 2}):
        frame(w, 3, frames=2, **kw)
    frame(W.arap_beam(8, 3, 3, seed=6), 3, lmax_scale=1.5)

    sim = frame(w, 2)
    h = sim.hier()
    rp, col, val = h.matrix(0)
    b = np.random.default_rng(1).standard_normal(rp.shape[0] - 1)
    h.vcycle(b)
    h.pcg(b, tol=1e-8, max_iters=100)
    for l in range(h.levels - 1):
        h.transfer(l)
        h.info(l)
    h.colors()
    h.refresh(val * 1.01)
    h.coarse_solve(np.ones(h.info(h.levels - 1)["n"]))
    own = O.Hier.build(rp, col, val, O.default_opts(n_cand=6))
    own.transfer_qr(0, 6)
    del own
    prio = np.arange(rp.shape[0] - 1, dtype=np.int64)[::-1].copy()
    O.aggregate(rp, col, val, prio)
    O.color(rp, col, prio)
    print("SANITIZED ORACLE OK")
""")


def _preload_in_use():
    return bool(os.environ.get("LD_PRELOAD")) or os.path.exists("/etc/ld.so.preload")


@pytest.mark.timeout(600)
def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    if _preload_in_use():
        pytest.skip("a library is already preloaded here; the ASan runtime must come first")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no ASan runtime")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fPIC", "-shared", "-o", lib, SRC, "-lm"])
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, MGPBD_ORACLE_LIB=lib, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=540)
    report = r.stdout[-4000:] + r.stderr[-8000:]
    assert r.returncode == 0, report
    assert "SANITIZED ORACLE OK" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
