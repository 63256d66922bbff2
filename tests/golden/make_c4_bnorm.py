"""Write the FP64 oracle's |b| history of the first frame of the stiff
ellipsoid (compliance 1e-12, dt 1/30, 30 % axial squeeze, no pins, no
gravity; copy 0 of the eight-copy stress batch) with a fixed number of PCG
iterations per solve, so that the GPU run can be compared with it global
iteration by global iteration (Algorithm 1: b = -C - alpha~ lambda of Eq. 3
at each iteration). Calls only the oracle. Two margins on the power-method
lambda_max: 1.5, with which the lazy setup (Sec. 4.2) keeps one hierarchy for
the whole frame, and the default 1.05, with which the V-cycle of this quickly
changing body stops being positive definite at iteration 5 and the frame sets
up afresh there (resetup_on_breakdown) and goes on.

    python tests/golden/make_c4_bnorm.py          (several minutes per margin, one core)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2505_13390_amd import workloads as W  # noqa: E402

N_ITERS = 20
FORCED = 20
RUNS = ((1.5, "c4_copy0_frame0_bnorm.txt"), (1.05, "c4_copy0_frame0_bnorm_lmax105.txt"))


def write(lmax_scale, name):
    out = os.path.join(HERE, name)
    w = W.stiff_c4(copies=1)[0]
    sim = O.Sim(w, O.default_opts(lmax_scale=lmax_scale))
    pos, vel = O.positions(w)
    t0 = time.time()
    r = sim.step(pos, vel, N_ITERS, force_pcg=[FORCED] * N_ITERS)
    assert r["status"] == 0, r["status"]
    with open(out, "w") as f:
        f.write("# FP64 oracle, stiff ellipsoid copy 0 (64x64x128 grid, 3,615,756 rows), "
                "frame 0,\n# lmax_scale %.2f, %d global iterations with %d forced PCG iterations each; "
                "|b| (Algorithm 1, Eq. 3), the final\n# recurrence |r|/|b| of each solve and whether "
                "the setup ran (1) or ran again after a\n# breakdown (2). Written by "
                "tests/golden/make_c4_bnorm.py.\n" % (lmax_scale, N_ITERS, FORCED))
        for k in range(N_ITERS):
            f.write("%d %.17e %.17e %d\n" % (k, r["bnorm"][k], r["ratio"][k], r["setup"][k]))
    print("wrote %s in %.0f s" % (out, time.time() - t0))
    print(np.array2string(r["bnorm"], precision=6), r["setup"].tolist())


def main():
    for lmax_scale, name in RUNS:
        if len(sys.argv) > 1 and name not in sys.argv[1:]:
            continue
        write(lmax_scale, name)


if __name__ == "__main__":
    main()
