"""The stiff large-step stress workload: the ellipsoid muscle with compliance
1e-12, dt 1/30, squeezed to 70 % along its long axis, free (no pins, no
gravity). Its first frame's |b| history (|b| = |-C - alpha~ lambda| of Eq. 3
at each global iteration of Algorithm 1) against the FP64 oracle's, written by
tests/golden/make_c4_bnorm.py with the same 20 forced PCG iterations per solve
and the same lmax_scale 1.5: as one body, and as body 0 of a batch of two
copies. Both sides start each solve from the same A and b only at iteration 0;
later iterations see positions that differ by the rounding of the previous
solves, so the history is compared to a bar derived from that (below). At
the default margin 1.05 the same frame breaks down at iteration 5 under the
hierarchy kept from iteration 0 and sets up afresh there, on both sides."""
import os

import numpy as np
import pytest

from paper_2505_13390_amd import workloads as W
from tests.conftest import GOLDEN
from tests.gpu_common import B, log, opts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_ITERS = 20
FORCED = 20
LMAX_SCALE = 1.5
# FP64: the forced solves agree with the oracle's to ~1e-12 relative in
# lambda at full size (tests/test_gpu_full_size_forced.py); the positions and
# so |b| of the next iteration inherit that, amplified by the unconverged,
# very stiff solves of the following iterations (compliance 1e-12: the
# preconditioned system's condition number is near 1e12). Observed at most
# 2.7e-9 (one body) and 2.9e-9 (batch), both at iteration 18; 1e-7 relative
# per iteration is about 35 times that.
FP64_BNORM = 1e-7


def golden(name="c4_copy0_frame0_bnorm.txt"):
    path = os.path.join(GOLDEN, name)
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    return np.array([float(r[1]) for r in rows]), np.array([float(r[2]) for r in rows])


def golden_setup(name):
    path = os.path.join(GOLDEN, name)
    return [int(l.split()[3]) for l in open(path) if not l.startswith("#")]


def _check(tag, bn, ref):
    rel = np.abs(bn - ref) / ref
    log("%s |b|: %s" % (tag, np.array2string(bn, precision=6, max_line_width=200)))
    log("%s relative difference: %s" % (tag, np.array2string(rel, precision=2,
                                                              max_line_width=200)))
    log("%s relative difference per iteration: max %.3e (iteration %d)"
        % (tag, rel.max(), int(rel.argmax())))
    assert bn.shape == ref.shape
    assert rel.max() <= FP64_BNORM


def test_c4_first_frame_bnorm_history():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref, ref_ratio = golden()
    w = W.stiff_c4(copies=1)[0]
    _, go = opts(lmax_scale=LMAX_SCALE)
    body = B.Body(w, go)
    B.mgpbd_force_pcg_iters(body.ctx, [FORCED] * N_ITERS)
    r = body.step(N_ITERS)
    assert (r["pcg_iters"] == FORCED).all()
    _check("C4 body", r["bnorm"], ref)
    body.close()


def test_c4_first_frame_bnorm_history_in_a_batch():
    """copies 0 and 1 as one batch (FP64); copy 0 against the same history"""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref, _ = golden()
    ws = W.stiff_c4(copies=2)
    _, go = opts(lmax_scale=LMAX_SCALE)
    batch = B.Batch(ws, go)
    for b in batch.bodies:
        B.mgpbd_force_pcg_iters(b.ctx, [FORCED] * N_ITERS)
    res = batch.step(N_ITERS)
    _check("C4 batch body 0", res[0]["bnorm"], ref)
    batch.close()


def test_c4_default_margin_sets_up_afresh_after_breakdown():
    """The same frame at the default margin 1.05: the hierarchy and omega
    kept from iteration 0 stop preconditioning A at iteration 5 and PCG breaks
    down; with resetup_on_breakdown (the default) both sides set up afresh at
    that iteration and go on. The setup flags must match the oracle's
    (tests/golden/c4_copy0_frame0_bnorm_lmax105.txt) and |b| of every
    iteration must stay within the bar above."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    name = "c4_copy0_frame0_bnorm_lmax105.txt"
    ref, _ = golden(name)
    ref_setup = golden_setup(name)
    assert 2 in ref_setup
    w = W.stiff_c4(copies=1)[0]
    _, go = opts()
    body = B.Body(w, go)
    B.mgpbd_force_pcg_iters(body.ctx, [FORCED] * N_ITERS)
    r = body.step(N_ITERS)
    log("C4 default margin: setup oracle %s gpu %s" % (ref_setup, r["setup_ran"].tolist()))
    assert r["setup_ran"].tolist() == ref_setup
    assert (r["pcg_iters"] == FORCED).all()
    _check("C4 body, default margin", r["bnorm"], ref)
    body.close()
