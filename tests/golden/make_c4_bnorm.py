"""Write the FP64 oracle's |b| history of the first frame of the stiff
ellipsoid (compliance 1e-12, dt 1/30, 30 % axial squeeze, no pins, no
gravity; copy 0 of the eight-copy stress batch) with a fixed number of PCG
iterations per solve, so that the GPU run can be compared with it global
iteration by global iteration (Algorithm 1: b = -C - alpha~ lambda of Eq. 3
at each iteration). Calls only the oracle. The Jacobi weights use
lmax_scale 1.5: the lazy setup (Sec. 4.2) keeps omega from iteration 0 while
this squeezed, nearly rigid body changes quickly within the frame, and at the
default 1.05 the V-cycle stops being positive definite at iteration 5.

    python tests/golden/make_c4_bnorm.py   (several minutes on one core)
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
LMAX_SCALE = 1.5
OUT = os.path.join(HERE, "c4_copy0_frame0_bnorm.txt")


def main():
    w = W.stiff_c4(copies=1)[0]
    sim = O.Sim(w, O.default_opts(lmax_scale=LMAX_SCALE))
    pos, vel = O.positions(w)
    t0 = time.time()
    r = sim.step(pos, vel, N_ITERS, force_pcg=[FORCED] * N_ITERS)
    assert r["status"] == 0, r["status"]
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, stiff ellipsoid copy 0 (64x64x128 grid, 3,615,756 rows), "
                "frame 0,\n# lmax_scale %.2f, %d global iterations with %d forced PCG iterations each; "
                "|b| (Algorithm 1, Eq. 3) then the final\n# recurrence |r|/|b| of each "
                "solve. Written by tests/golden/make_c4_bnorm.py.\n" % (LMAX_SCALE, N_ITERS, FORCED))
        for k in range(N_ITERS):
            f.write("%d %.17e %.17e\n" % (k, r["bnorm"][k], r["ratio"][k]))
    print("wrote %s in %.0f s" % (OUT, time.time() - t0))
    print(np.array2string(r["bnorm"], precision=6))


if __name__ == "__main__":
    main()
