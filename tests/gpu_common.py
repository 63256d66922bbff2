"""Shared helpers of the GPU parity tests: run one workload through the HIP
library (via the C ABI binding) and through the FP64 CPU oracle."""
import sys

import numpy as np

from oracle import oracle as O
from paper_2505_13390_amd import binding as B
from paper_2505_13390_amd import workloads as W

COMMON = ("theta", "gs_sweeps", "pre_sweeps", "post_sweeps", "lambda_min", "coarse_max",
          "dense_max", "max_levels", "power_iters", "omega_relax", "tol", "max_pcg", "seed",
          "reuse_interval", "b_mode", "eps_b", "lmax_scale", "smoother", "n_cand", "power_max",
          "power_tol", "resetup_on_breakdown")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def opts(**kw):
    """Matching (oracle, gpu) options; gpu-only keys: precision, use_graph,
    check_every, profile_spmv, spmv_tile, spmv_lanes, matrix_free, vcycle_tail,
    fuse_transfers."""
    gkw = {k: kw.pop(k) for k in list(kw) if k in ("precision", "use_graph", "check_every",
                                                   "profile_spmv", "spmv_tile", "spmv_lanes",
                                                   "matrix_free", "vcycle_tail",
                                                   "fuse_transfers")}
    o = O.default_opts(**kw)
    if gkw.get("precision", 0) == B.PREC_MIXED:
        o.flexible = 1
    g = B.mgpbd_default_options(**kw, **gkw)
    for k in COMMON:
        assert getattr(o, k) == getattr(g, k), k
    return o, g


def rel_pos_err(x, xref):
    """max |x - x_ref| / max |x_ref| over all components"""
    return float(np.abs(x - xref).max() / np.abs(xref).max())


def run_both(w, n_iters, frames=1, force_from_oracle=False, **kw):
    oo, go = opts(**kw)
    sim = O.Sim(w, oo)
    body = B.Body(w, go)
    pos, vel = O.positions(w)
    ores, gres = [], []
    for f in range(frames):
        r = sim.step(pos, vel, n_iters)
        ores.append(r)
        if force_from_oracle:
            B.mgpbd_force_pcg_iters(body.ctx, r["pcg_iters"])
        gres.append(body.step(n_iters))
    return sim, body, pos, vel, ores, gres
