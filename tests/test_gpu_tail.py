"""The fused coarse end of the V-cycle (Sec. 4.4-4.5): one launch per V-cycle
runs every level on which each body has at most vcycle_tail rows, one
workgroup per body. It sums in the order of the per-level kernels, so a frame
with it must equal, bit for bit, the same frame with one launch per pass
(vcycle_tail = 0), in FP64 and with the FP32 V-cycle, with the Jacobi and
Chebyshev smoothers, for one body and for a batch (both with the separate
transfer kernels, fuse_transfers = 0, whose order it follows). It is off by default
(slower than the per-level launches on the workloads measured), so these
tests switch it on."""
import numpy as np
import pytest

from paper_2505_13390_amd import workloads as W
from tests.gpu_common import B, log, opts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAIL = 2048   # rows per body at or below which the coarse levels are fused


def _beam():
    return W.beam(64, 16, 16, seed=11, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9)


def _same(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _tail_start(ctx, limit):
    """first level from which on every level has at most limit rows (one body)"""
    L = B.mgpbd_num_levels(ctx)
    sizes = [B.mgpbd_get_level(ctx, l)["n"] for l in range(L)]
    l0 = L
    for l in range(L - 1, 0, -1):
        if sizes[l] > limit:
            break
        l0 = l
    return l0, sizes


@pytest.mark.parametrize("kind", ["fp64", "mixed", "chebyshev", "arap"])
def test_tail_matches_per_level_passes(kind):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kw = {"fp64": {}, "mixed": {"precision": B.PREC_MIXED}, "chebyshev": {"smoother": 1},
          "arap": {"lmax_scale": 1.5}}[kind]
    kw["fuse_transfers"] = 0
    w = W.arap_a0() if kind == "arap" else _beam()
    _, g0 = opts(vcycle_tail=0, **kw)
    ref = B.Body(w, g0)
    r0 = ref.step(3)
    _, g1 = opts(vcycle_tail=TAIL, **kw)
    fused = B.Body(w, g1)
    B.mgpbd_force_pcg_iters(fused.ctx, r0["pcg_iters"])
    r1 = fused.step(3)
    l0, sizes = _tail_start(fused.ctx, g1.vcycle_tail)
    log("%s: levels %s, fused from level %d, pcg iters %s / %s" % (
        kind, sizes, l0, r0["pcg_iters"].tolist(), r1["pcg_iters"].tolist()))
    assert 1 <= l0 < len(sizes)
    assert (r1["pcg_iters"] == r0["pcg_iters"]).all()
    assert _same(fused.positions(), ref.positions())
    assert _same(fused.velocities(), ref.velocities())
    assert _same(B.mgpbd_get_lambda(fused.ctx, fused.m), B.mgpbd_get_lambda(ref.ctx, ref.m))
    # with per-level timing, every level below the start of the tail has no
    # passes of its own: the tail's one launch is timed on its first level
    _, g2 = opts(profile_spmv=1, vcycle_tail=TAIL, **kw)
    prof = B.Body(w, g2)
    B.mgpbd_force_pcg_iters(prof.ctx, r0["pcg_iters"])
    r2 = prof.step(3)
    ms = r2["ms_level"][:len(sizes)]
    log("  per-level ms over %d V-cycles: %s" % (r2["vcycles"], ["%.2f" % v for v in ms]))
    assert r2["vcycles"] > 0
    assert all(v > 0 for v in ms[:l0 + 1]) and all(v == 0 for v in ms[l0 + 1:])
    assert _same(prof.positions(), ref.positions())
    for b in (ref, fused, prof):
        b.close()


def test_tail_batch_matches_per_level_passes():
    """a batch of beams of uneven size (one workgroup per body in the tail),
    FP32 V-cycle as the batch workload runs it"""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ws = [W.beam(4 * n, n, n, seed=40 + n, volumes=True, alpha_edge=1e-8, alpha_vol=1e-8)
          for n in (4, 7, 10, 13, 16)]
    _, g0 = opts(vcycle_tail=0, precision=B.PREC_MIXED, fuse_transfers=0)
    ref = B.Batch(ws, g0)
    r0 = ref.step(2)
    _, g1 = opts(precision=B.PREC_MIXED, vcycle_tail=TAIL, fuse_transfers=0)
    fused = B.Batch(ws, g1)
    for b, r in zip(fused.bodies, r0):
        B.mgpbd_force_pcg_iters(b.ctx, r["pcg_iters"])
    r1 = fused.step(2)
    for k in range(len(ws)):
        log("body %d: pcg iters %s / %s" % (k, r0[k]["pcg_iters"].tolist(),
                                             r1[k]["pcg_iters"].tolist()))
        assert (r1[k]["pcg_iters"] == r0[k]["pcg_iters"]).all()
        assert _same(fused.bodies[k].positions(), ref.bodies[k].positions())
        assert _same(fused.bodies[k].velocities(), ref.bodies[k].velocities())
    ref.close()
    fused.close()
