"""GPU parity of batching: several uneven bodies stepped as one block-diagonal
system (one launch per kernel for all bodies) against each body's own FP64
CPU oracle run. Per body, the first setup is bit-exact (pattern, aggregates,
colours, candidates, P and every coarse level's values, with the indices
shifted by the body's offsets) and positions agree within 1e-9 relative."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_13390_amd import workloads as W
from tests.gpu_common import B, log, opts, rel_pos_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


CMAX = 60   # coarse_max small enough for three hierarchy depths at test sizes


def bodies():
    """Uneven members: one, two and three levels (one body small enough to be
    solved densely on level 0), one without volume rows, perturbed starts."""
    return [
        W.perturbed(W.beam(24, 4, 4, seed=11, volumes=True, alpha_edge=1e-6, alpha_vol=1e-6,
                           name="b24"), 2e-3, seed=1),
        W.tiny_beam(2, 1, 1, seed=12),
        W.perturbed(W.beam(12, 3, 3, seed=13, volumes=True, alpha_edge=1e-7, alpha_vol=1e-7,
                           name="b12"), 1e-3, seed=2),
        W.beam(10, 2, 2, seed=14, volumes=False, alpha_edge=1e-6, name="b10e"),
        W.perturbed(W.beam(32, 4, 4, seed=15, volumes=True, alpha_edge=1e-6, alpha_vol=1e-6,
                           name="b32"), 1e-3, seed=3),
    ]


def run_batch(ws, n_iters, frames=1, force_from_oracle=False, **kw):
    oo, go = opts(coarse_max=CMAX, **kw)
    sims = [O.Sim(w, oo) for w in ws]
    states = [O.positions(w) for w in ws]
    batch = B.Batch(ws, go)
    ores, gres = [], []
    for f in range(frames):
        o = [s.step(p, v, n_iters) for s, (p, v) in zip(sims, states)]
        if force_from_oracle:
            for b, r in zip(batch.bodies, o):
                B.mgpbd_force_pcg_iters(b.ctx, r["pcg_iters"])
        ores.append(o)
        gres.append(batch.step(n_iters))
    return sims, states, batch, ores, gres


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def test_batch_first_setup_bit_exact_per_body():
    ws = bodies()
    sims, states, batch, ores, gres = run_batch(ws, 1)
    hs = [s.hier() for s in sims]
    depth = [h.levels for h in hs]
    log("per-body levels", depth, "rows", [s.m for s in sims])
    assert len(set(depth)) >= 3, "the batch should mix coarsening depths"
    ctx = batch.ctx
    L = B.mgpbd_num_levels(ctx)
    assert L == max(depth)
    for l in range(L):
        members = [k for k in range(len(ws)) if depth[k] > l]
        info = B.mgpbd_get_level(ctx, l)
        grp, gcol, gval = B.mgpbd_get_matrix(ctx, l)
        n_exp = sum(hs[k].info(l)["n"] for k in members)
        assert info["n"] == n_exp
        has_next = l + 1 < L
        if has_next:
            gagg = B.mgpbd_get_aggregates(ctx, l)
            gp, gB = B.mgpbd_get_transfer(ctx, l)
        r0 = a0 = 0
        for k in members:
            oi = hs[k].info(l)
            n = oi["n"]
            orp, ocol, oval = hs[k].matrix(l)
            e0 = grp[r0]
            assert np.array_equal(grp[r0:r0 + n + 1] - e0, orp), (l, k)
            assert np.array_equal(gcol[e0:e0 + oi["nnz"]] - r0, ocol), (l, k)
            assert same_bits(gval[e0:e0 + oi["nnz"]], oval), "level %d body %d values" % (l, k)
            coarsens = depth[k] > l + 1
            if has_next:
                seg = gagg[r0:r0 + n]
                if coarsens:
                    oagg, op, oB = hs[k].transfer(l)
                    na = int(oagg.max()) + 1
                    exp = np.where(oagg >= 0, oagg + a0, -1)
                    assert np.array_equal(seg, exp), "level %d body %d aggregates" % (l, k)
                    assert same_bits(gp[r0:r0 + n], op), "level %d body %d P" % (l, k)
                    assert same_bits(gB[r0:r0 + n], oB), "level %d body %d candidate" % (l, k)
                    a0 += na
                else:
                    assert (seg == -1).all(), "a body ending on level %d joined aggregates" % l
            r0 += n
        if has_next:
            assert a0 == info["n_agg"]
    # level-0 colours of every body that coarsens
    gc, _ = B.mgpbd_get_colors(ctx, sum(s.m for s in sims))
    r0 = 0
    for k, s in enumerate(sims):
        if depth[k] > 1:
            oc, _ = hs[k].colors()
            assert np.array_equal(gc[r0:r0 + s.m], oc), "body %d colours" % k
        r0 += s.m
    batch.close()


def test_batch_frames_match_each_body_oracle():
    ws = bodies()
    sims, states, batch, ores, gres = run_batch(ws, 6, frames=2)
    for k, (w, (pos, vel)) in enumerate(zip(ws, states)):
        err = rel_pos_err(batch.bodies[k].positions(), pos)
        log("body %d (%s): oracle iters %s gpu %s pos err %.3e" % (
            k, w.name, ores[-1][k]["pcg_iters"].tolist(), gres[-1][k]["pcg_iters"].tolist(), err))
        assert err <= 1e-9, k
        assert (gres[-1][k]["pcg_ratio"] <= 1e-6).all()
        assert gres[0][k]["setup_ran"][0] == 1 and gres[1][k]["setup_ran"][0] == 0
    batch.close()


def test_batch_with_forced_counts():
    ws = bodies()
    sims, states, batch, ores, gres = run_batch(ws, 5, force_from_oracle=True)
    for k, (pos, vel) in enumerate(states):
        assert (gres[0][k]["pcg_iters"] == ores[0][k]["pcg_iters"]).all()
        err = rel_pos_err(batch.bodies[k].positions(), pos)
        verr = float(np.abs(batch.bodies[k].velocities() - vel).max()
                     / max(np.abs(vel).max(), 1e-300))
        log("forced body %d: pos err %.3e vel err %.3e" % (k, err, verr))
        assert err <= 1e-9
    batch.close()


def test_batch_equals_separate_contexts_to_rounding():
    """The same bodies stepped one by one on the GPU: same hierarchy depth and
    PCG counts within rounding of the reductions, positions within 1e-10."""
    ws = bodies()
    _, go = opts(coarse_max=CMAX)
    single = [B.Body(w, go) for w in ws]
    sres = [b.step(4) for b in single]
    batch = B.Batch(ws, go)
    bres = batch.step(4)
    for k in range(len(ws)):
        a, b = sres[k]["pcg_iters"], bres[k]["pcg_iters"]
        assert np.abs(a.astype(int) - b.astype(int)).max() <= max(2, 0.05 * a.max()), (a, b)
        err = rel_pos_err(batch.bodies[k].positions(), single[k].positions())
        log("body %d: batch vs single iters %s %s pos diff %.3e" % (k, a.tolist(), b.tolist(), err))
        assert err <= 1e-10
        single[k].close()
    batch.close()


def test_batch_mixed_precision():
    ws = bodies()
    _, go = opts(precision=B.PREC_MIXED, coarse_max=CMAX)
    oo64, _ = opts(coarse_max=CMAX)
    batch = B.Batch(ws, go)
    res = batch.step(6)
    for k, w in enumerate(ws):
        sim = O.Sim(w, oo64)
        pos, vel = O.positions(w)
        sim.step(pos, vel, 6)
        err = rel_pos_err(batch.bodies[k].positions(), pos)
        log("mixed body %d: iters %s err %.3e" % (k, res[k]["pcg_iters"].tolist(), err))
        assert (res[k]["pcg_ratio"] <= 1e-6).all()
        assert err <= 1e-7
    batch.close()


def test_batch_eps_b_stops_bodies_independently():
    ws = bodies()
    o0, _ = opts(coarse_max=CMAX)
    probe = []
    for w in ws:
        s = O.Sim(w, o0)
        p, v = O.positions(w)
        probe.append(s.step(p, v, 6)["bnorm"])
    # a threshold between two iterations of body 0, far from every body's |b|
    eps = float(np.sqrt(probe[0][2] * probe[0][3]))
    allb = np.concatenate(probe)
    margin = np.abs(np.log(allb / eps)).min()
    log("eps_b %.6e, closest |b| ratio margin %.3e" % (eps, margin))
    if margin < 1e-6:
        pytest.skip("a body's |b| lies too close to the threshold")
    sims, states, batch, ores, gres = run_batch(ws, 6, eps_b=eps)
    done = [r["iters_done"] for r in gres[0]]
    # the oracle stops a body after the first iteration whose |b| < eps_b
    odone = []
    for r in ores[0]:
        below = np.nonzero(r["bnorm"] < eps)[0]
        odone.append(int(below[0]) + 1 if below.size else 6)
    log("iterations done: gpu", done, "oracle", odone)
    assert done == odone
    assert len(set(done)) >= 2
    for k, (pos, vel) in enumerate(states):
        assert rel_pos_err(batch.bodies[k].positions(), pos) <= 1e-9
    batch.close()


def test_batch_rejects_mismatched_members():
    a = W.tiny_beam(3, 1, 1)
    b = W.tiny_beam(4, 1, 1)
    b.dt = a.dt / 2
    ba, bb = B.Body(a), B.Body(b)
    with pytest.raises(B.MgpbdError):
        B.mgpbd_batch_create([ba.ctx, bb.ctx])
    ba.close()
    bb.close()


def test_apply_on_a_batch_context():
    """mgpbd_apply on the batch's system context: all bodies' rows back to
    back, equal to the block-diagonal assembled matrix up to summation order."""
    import scipy.sparse as sp
    ws = bodies()
    _, go = opts(coarse_max=CMAX)
    batch = B.Batch(ws, go)
    batch.step(1)
    rp, col, val = B.mgpbd_get_matrix(batch.ctx, 0)
    A = sp.csr_matrix((val, col, rp))
    m = rp.size - 1
    assert m == sum(w.n_rows for w in ws)
    x = np.random.default_rng(9).standard_normal(m)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    yt = torch.empty_like(xt)
    B.mgpbd_apply(batch.ctx, xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    err = float((np.abs(y - A @ x) / (abs(A) @ np.abs(x))).max())
    log("batch apply: %d rows, max row error %.3e of |A||x|" % (m, err))
    batch.close()
    assert err <= 1e-13


def empty_body(seed):
    """A body with vertices but no constraint rows (all rows removed)."""
    w = W.tiny_beam(3, 2, 1, seed=seed)
    w.edges = np.zeros((0, 2), np.int32)
    w.vol_tet = np.zeros(0, np.int32)
    w.alpha = np.zeros(0)
    w.name = "empty"
    return w


@pytest.mark.parametrize("mf,smoother", [(1, 0), (0, 0), (1, 1)])
def test_batch_with_a_body_without_constraints(mf, smoother):
    """A member without rows sits in the batch as an empty segment: it takes
    the semi-implicit Euler step of Algorithm 1 (bit for bit, as in the
    oracle) while the other members solve as before (forced counts, 1e-9)."""
    ws = bodies()[:3]
    ws.insert(1, empty_body(21))
    sims, states, batch, ores, gres = run_batch(ws, 4, frames=2, force_from_oracle=True,
                                                matrix_free=mf, smoother=smoother)
    for k, (w, (pos, vel)) in enumerate(zip(ws, states)):
        if w.n_rows == 0:
            assert (gres[-1][k]["pcg_iters"] == 0).all()
            assert np.array_equal(batch.bodies[k].positions(), pos)
            assert np.array_equal(batch.bodies[k].velocities(), vel)
            log("empty member %d: Euler step bit-exact" % k)
            continue
        assert (gres[-1][k]["pcg_iters"] == ores[-1][k]["pcg_iters"]).all()
        err = rel_pos_err(batch.bodies[k].positions(), pos)
        log("member %d (%s, mf %d, smoother %d): pos err %.3e" % (k, w.name, mf, smoother, err))
        assert err <= 1e-9
    batch.close()


def test_batch_of_bodies_without_constraints():
    ws = [empty_body(22), empty_body(23)]
    sims, states, batch, ores, gres = run_batch(ws, 3, frames=2)
    for k, (pos, vel) in enumerate(states):
        assert np.array_equal(batch.bodies[k].positions(), pos)
        assert np.array_equal(batch.bodies[k].velocities(), vel)
    batch.close()
