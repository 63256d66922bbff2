"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs. Integer and index results (pattern, aggregates,
colours) must be bit-exact; the setup is a pure function of the bits of A,
so the FP64 values that feed it (A, candidates, P, Galerkin products) are
compared bitwise too; positions must agree within 1e-9 relative (FP64)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_13390_amd import workloads as W
from tests.gpu_common import B, log, opts, rel_pos_err, run_both

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield


def test_device_sqrt_and_division_are_correctly_rounded():
    rng = np.random.default_rng(0)
    n = 1 << 20
    a = np.abs(rng.standard_normal(n)) * np.exp2(rng.integers(-300, 300, n).astype(float))
    b = rng.standard_normal(n) * np.exp2(rng.integers(-300, 300, n).astype(float))
    special = np.array([1.0, 2.0, 3.0, 4.0, 0.25, 1e-310, 5e-324, 1.7976931348623157e308,
                        0.0, 9007199254740993.0, 1.0000000000000002, 0.9999999999999999])
    a[:special.size] = special
    b[:special.size] = special[::-1] + 1.0
    ta = torch.tensor(a, device="cuda")
    tb = torch.tensor(b, device="cuda")
    s, q = B.mgpbd_selftest_sqrt_div(ta, tb)
    s, q = s.cpu().numpy(), q.cpu().numpy()
    assert np.array_equal(s.view(np.uint64), np.sqrt(a).view(np.uint64))
    assert np.array_equal(q.view(np.uint64), (a / b).view(np.uint64))


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def close(a, b, rtol):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max(initial=0.0) <= rtol * max(np.abs(b).max(initial=0.0), 1e-300)


def compare_hierarchy(sim, body, what, exact=True):
    """Setup built by both sides. Patterns, aggregates and colours always
    bit-exact. exact: the setup saw bit-identical A (first global iteration),
    so candidates, P and every level's values are bitwise equal; otherwise the
    values (of a later iteration) agree to 1e-9 relative."""
    h = sim.hier()
    L = B.mgpbd_num_levels(body.ctx)
    log(what, "levels oracle", h.levels, "gpu", L)
    assert L == h.levels
    for l in range(L):
        gi = B.mgpbd_get_level(body.ctx, l)
        oi = h.info(l)
        log("  level", l, "n", gi["n"], "nnz", gi["nnz"], "omega gpu %.12g oracle %.12g"
            % (gi["omega"], oi["omega"]))
        assert gi["n"] == oi["n"] and gi["nnz"] == oi["nnz"]
        grp, gcol, gval = B.mgpbd_get_matrix(body.ctx, l)
        orp, ocol, oval = h.matrix(l)
        assert np.array_equal(grp, orp) and np.array_equal(gcol, ocol)
        if exact:
            nbad = int((gval.view(np.uint64) != oval.view(np.uint64)).sum())
            assert nbad == 0, "level %d: %d matrix values differ" % (l, nbad)
        else:
            assert close(gval, oval, 1e-9), "level %d values" % l
        if oi["omega"] > 0:
            assert abs(gi["omega"] - oi["omega"]) <= 1e-6 * oi["omega"]
        if l + 1 < L:
            assert gi["n_agg"] == h.info(l + 1)["n"]
            gagg = B.mgpbd_get_aggregates(body.ctx, l)
            oagg, op, oB = h.transfer(l)
            assert np.array_equal(gagg, oagg), "level %d aggregates differ" % l
            gp, gB = B.mgpbd_get_transfer(body.ctx, l)
            if exact:
                assert same_bits(gB, oB), "candidate differs"
                assert same_bits(gp, op), "P differs"
            else:
                assert close(gB, oB, 1e-6) and close(gp, op, 1e-6)
    if h.levels > 1 and h.info(0)["n_colors"] > 0:
        oc, onc = h.colors()
        gc, gnc = B.mgpbd_get_colors(body.ctx, sim.m)
        assert gnc == onc and np.array_equal(gc, oc)


def iters_close(a, b):
    """Long PCG runs (hundreds of iterations) amplify rounding differences, so
    the two sides may cross the tolerance a few percent apart; both must
    satisfy it (checked separately)."""
    a, b = int(a), int(b)
    return abs(a - b) <= max(3, 0.15 * max(a, b))


def true_residual(body, sim):
    """|A dlambda - b| / |b| of the GPU's first solve (lambda = dlambda after one
    global iteration), with the GPU's own A and b."""
    import scipy.sparse as sp
    rp, col, val = B.mgpbd_get_matrix(body.ctx, 0)
    A = sp.csr_matrix((val, col, rp))
    b = B.mgpbd_get_rhs(body.ctx, sim.m)
    x = B.mgpbd_get_lambda(body.ctx, sim.m)
    return float(np.linalg.norm(A @ x - b) / np.linalg.norm(b))


def test_c0_first_iteration_assembly_and_setup_bit_exact():
    w = W.beam_c0()
    log("C0 rows", w.n_rows)
    sim, body, pos, vel, ores, gres = run_both(w, 1)
    assert ores[0]["status"] == 0
    # A pattern and values at iteration 0 (same predicted positions)
    orp, ocol = sim.pattern()
    grp, gcol, gval = B.mgpbd_get_matrix(body.ctx, 0)
    assert np.array_equal(grp, orp) and np.array_equal(gcol, ocol)
    assert np.array_equal(gval.view(np.uint64), sim.matrix_values().view(np.uint64))
    assert np.array_equal(B.mgpbd_get_rhs(body.ctx, sim.m).view(np.uint64),
                          sim.rhs().view(np.uint64))
    compare_hierarchy(sim, body, "C0")
    log("pcg iters oracle", ores[0]["pcg_iters"], "gpu", gres[0]["pcg_iters"])
    assert iters_close(ores[0]["pcg_iters"][0], gres[0]["pcg_iters"][0])
    tr = true_residual(body, sim)
    log("true relative residual of the GPU solve %.3e" % tr)
    assert tr <= 1.5e-6
    err = rel_pos_err(body.positions(), pos)
    log("C0 1-iteration position error", err)
    assert err <= 1e-9


@pytest.mark.parametrize("mf", [1, 0])
def test_c0_frame_positions_within_1e9(mf):
    """Fine-level products matrix-free (default) or from the assembled CSR."""
    w = W.beam_c0()
    sim, body, pos, vel, ores, gres = run_both(w, 20, matrix_free=mf)
    log("oracle iters", ores[0]["pcg_iters"].tolist())
    log("gpu    iters", gres[0]["pcg_iters"].tolist())
    err = rel_pos_err(body.positions(), pos)
    verr = float(np.abs(body.velocities() - vel).max() / max(np.abs(vel).max(), 1e-300))
    lerr = float(np.abs(B.mgpbd_get_lambda(body.ctx, sim.m) - sim.lam()).max()
                 / np.abs(sim.lam()).max())
    log("C0 frame (matrix_free=%d): position err %.3e velocity err %.3e lambda err %.3e"
        % (mf, err, verr, lerr))
    assert err <= 1e-9
    assert (gres[0]["pcg_ratio"] <= 1e-6).all()


def test_c0_frame_with_forced_pcg_counts():
    """Parity mode: both sides run exactly the oracle's PCG iteration counts."""
    w = W.beam_c0()
    sim, body, pos, vel, ores, gres = run_both(w, 20, force_from_oracle=True)
    assert (gres[0]["pcg_iters"] == ores[0]["pcg_iters"]).all()
    err = rel_pos_err(body.positions(), pos)
    log("C0 forced-count position error %.3e" % err)
    assert err <= 1e-9


@pytest.mark.parametrize("tile,lanes", [(1024, 0), (2048, 0), (4096, 0), (-1, 4), (-1, 64),
                                        (-2, 0)])
def test_csr_pass_variants_match_oracle(tile, lanes):
    """Every CSR product variant the autotuner may pick (LDS stream tiles,
    lanes-per-row counts, SELL-C-sigma with tile -2) gives oracle parity on the
    8x8x32 beam. The GPU runs the oracle's PCG counts: this beam's solves end
    on a residual plateau near 1e-6, where rounding-level differences move the
    stopping iteration by up to 20 (e.g. 461 against 480), and the matrix of
    the next iteration then differs by that solve's 1e-6 tolerance rather than
    by rounding."""
    w = W.beam_c0()
    sim, body, pos, vel, ores, gres = run_both(w, 3, force_from_oracle=True, spmv_tile=tile,
                                               spmv_lanes=lanes, matrix_free=0)
    compare_hierarchy(sim, body, "tile %d lanes %d" % (tile, lanes), exact=False)
    err = rel_pos_err(body.positions(), pos)
    log("  position error %.3e iters %s %s" % (err, ores[0]["pcg_iters"].tolist(),
                                              gres[0]["pcg_iters"].tolist()))
    assert err <= 1e-9


def test_graph_and_direct_launch_are_bitwise_identical():
    w = W.tiny_beam(12, 4, 4, volumes=True, alpha_edge=1e-8, alpha_vol=1e-8)
    res = []
    for g in (1, 0, 1):
        _, go = opts(use_graph=g, coarse_max=60)
        body = B.Body(w, go)
        body.step(4)
        res.append(body.positions())
        body.close()
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])


@pytest.mark.parametrize("dims,vols,cmax", [((1, 1, 1), False, 400), ((2, 1, 1), True, 400),
                                            ((5, 3, 2), True, 40), ((9, 2, 3), True, 25),
                                            ((16, 4, 4), True, 400), ((20, 6, 5), False, 120)])
def test_small_and_ragged_meshes(dims, vols, cmax):
    w = W.tiny_beam(*dims, volumes=vols, alpha_edge=1e-7, alpha_vol=1e-8)
    log("mesh", dims, "rows", w.n_rows)
    sim, body, pos, vel, ores, gres = run_both(w, 5, coarse_max=cmax)
    assert ores[0]["status"] == 0
    compare_hierarchy(sim, body, str(dims), exact=False)
    err = rel_pos_err(body.positions(), pos)
    log("  position error %.3e" % err, "iters", ores[0]["pcg_iters"].tolist(),
        gres[0]["pcg_iters"].tolist())
    assert err <= 1e-9


def test_lazy_setup_schedule_and_parity_over_frames():
    w = W.tiny_beam(16, 4, 4, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9)
    sim, body, pos, vel, ores, gres = run_both(w, 4, frames=3, reuse_interval=2, coarse_max=80)
    for o, g in zip(ores, gres):
        assert (o["setup"] == g["setup_ran"]).all()
    assert [g["setup_ran"].tolist() for g in gres] == [[1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0]]
    err = rel_pos_err(body.positions(), pos)
    log("3 frames lazy: position error %.3e" % err)
    assert err <= 1e-9


def test_setup_every_iteration_mode():
    w = W.tiny_beam(10, 3, 3, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9)
    sim, body, pos, vel, ores, gres = run_both(w, 3, reuse_interval=0, coarse_max=40)
    assert gres[0]["setup_ran"].tolist() == [1, 1, 1]
    compare_hierarchy(sim, body, "every-iteration", exact=False)
    assert rel_pos_err(body.positions(), pos) <= 1e-9


def test_solve_entry_matches_oracle():
    w = W.perturbed(W.tiny_beam(12, 4, 4, volumes=True, alpha_edge=1e-8, alpha_vol=1e-8), 0.01)
    sim = O.Sim(w)
    val, b = sim.assemble(w.x0)
    rp, col = sim.pattern()
    oo, go = opts(coarse_max=60)
    h = O.Hier.build(rp, col, val, oo)
    xo, st = h.pcg(b, 1e-8, 1000)
    ctx = B.mgpbd_solver_create(go)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    xg = torch.zeros(sim.m, dtype=torch.float64, device="cuda")
    r = B.mgpbd_solve(ctx, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.float64),
                      dev(b, torch.float64), 1e-8, xg)
    log("solve iters oracle", st["iters"], "gpu", r["iters"])
    assert r["status"] == B.OK
    for l in range(h.levels - 1):
        assert np.array_equal(B.mgpbd_get_aggregates(ctx, l), h.transfer(l)[0])
    x = xg.cpu().numpy()
    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, rp))
    # the recurrence residual stops at 1e-8; the true residual may drift from
    # it by rounding (a few ulps of |A||x| per iteration), far below 1e-8 here
    true_ratio = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    log("solve: recurrence ratio %.3e, true ratio %.3e" % (r["ratio"], true_ratio))
    assert r["ratio"] <= 1e-8 and true_ratio <= 2e-8
    assert iters_close(r["iters"], st["iters"])
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()
    B.mgpbd_destroy(ctx)


def test_solve_rejects_malformed_csr():
    """mgpbd_solve checks the caller's CSR on the device before any kernel
    indexes through it: non-monotone row bounds, rowptr[0] != 0, a column
    outside [0, n) and repeated columns are E_INVALID_ARG."""
    w = W.tiny_beam(3, 1, 1)
    sim = O.Sim(w)
    val, b = sim.assemble(w.x0)
    rp, col = sim.pattern()
    n = sim.m
    ctx = B.mgpbd_solver_create(opts()[1])
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    xg = torch.zeros(n, dtype=torch.float64, device="cuda")
    bad = []
    r1 = rp.copy(); r1[2], r1[3] = r1[3], r1[2]           # decreasing bounds
    bad.append(("decreasing rowptr", r1, col))
    r2 = rp.copy(); r2[0] = 1                              # rowptr[0] != 0
    bad.append(("rowptr[0] = 1", r2, col))
    c1 = col.copy(); c1[rp[1] - 1] = n                     # column == n
    bad.append(("column n", rp, c1))
    c2 = col.copy(); c2[rp[1] + 1] = c2[rp[1]]             # repeated column
    bad.append(("repeated column", rp, c2))
    for what, r, c in bad:
        with pytest.raises(B.MgpbdError) as e:
            B.mgpbd_solve(ctx, dev(r, torch.int64), dev(c, torch.int32), dev(val, torch.float64),
                          dev(b, torch.float64), 1e-8, xg)
        log("%s: %s" % (what, e.value))
        assert e.value.status == B.E_INVALID_ARG, what
    # the context still solves a valid matrix afterwards
    res = B.mgpbd_solve(ctx, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.float64),
                        dev(b, torch.float64), 1e-8, xg)
    assert res["status"] == B.OK
    B.mgpbd_destroy(ctx)


@pytest.mark.parametrize("mf,tile", [(1, 0), (0, 0), (0, -2), (2, 0)])
def test_mixed_precision_against_fp64_oracle(mf, tile):
    """FP32 V-cycle against the FP64 oracle: matrix-free, assembled or timed
    choice (mf 2) of the fine-level operator, and every level in the
    SELL-C-sigma format (tile -2)."""
    w = W.beam_c0()
    oo, go = opts(precision=B.PREC_MIXED, matrix_free=mf, spmv_tile=tile)
    oo64, _ = opts()
    sim = O.Sim(w, oo64)
    pos, vel = O.positions(w)
    ro = sim.step(pos, vel, 20)
    body = B.Body(w, go)
    rg = body.step(20)
    err = rel_pos_err(body.positions(), pos)
    log("mixed C0: position error vs FP64 oracle %.3e" % err)
    log("iters fp64 oracle", ro["pcg_iters"].tolist())
    log("iters mixed gpu  ", rg["pcg_iters"].tolist())
    assert (rg["pcg_ratio"] <= 1e-6).all()
    assert err <= 1e-7


def test_rest_state_stays_bitwise_at_rest():
    w = W.tiny_beam(6, 2, 2, volumes=True)
    w.gravity = (0.0, 0.0, 0.0)
    _, go = opts()
    body = B.Body(w, go)
    x0 = body.positions()
    r = body.step(3)
    assert np.array_equal(body.positions(), x0)
    assert not body.velocities().any()
    assert (r["bnorm"] == 0).all() and (r["pcg_iters"] == 0).all()


def test_non_finite_positions_rejected_state_unchanged():
    w = W.tiny_beam(3, 1, 1)
    _, go = opts()
    body = B.Body(w, go)
    body.x[1][2] = float("nan")
    with pytest.raises(B.MgpbdError) as e:
        body.step(2)
    assert e.value.status == B.E_INVALID_ARG
    body.x[1][2] = 0.5
    body.step(1)


def test_create_rejects_bad_input():
    w = W.tiny_beam(2, 1, 1)
    _, go = opts()
    bad = w.alpha.copy()
    bad[0] = -1.0
    with pytest.raises(B.MgpbdError):
        B.mgpbd_create(w.rest, w.inv_mass, w.tets, w.edges, w.vol_tet, bad, w.dt, w.gravity, go)
    with pytest.raises(B.MgpbdError):
        B.mgpbd_create(w.rest, w.inv_mass, w.tets, w.edges[::-1], w.vol_tet, w.alpha, w.dt,
                       w.gravity, go)
    flipped = w.tets.copy()
    flipped[:, [1, 2]] = flipped[:, [2, 1]]
    with pytest.raises(B.MgpbdError):
        B.mgpbd_create(w.rest, w.inv_mass, flipped, w.edges, w.vol_tet, w.alpha, w.dt,
                       w.gravity, go)


@pytest.mark.parametrize("smoother,mf", [(1, 1), (1, 0), (2, 1), (2, 0)])
def test_other_smoothers_against_oracle(smoother, mf):
    """Sec. 4.5's Chebyshev (1) and multicolour Gauss-Seidel (2) smoothers, 2
    sweeps before and after, with both fine operators: positions within 1e-9
    of the oracle running the same smoother."""
    w = W.beam_c0()
    sim, body, pos, vel, ores, gres = run_both(w, 8, smoother=smoother, matrix_free=mf)
    err = rel_pos_err(body.positions(), pos)
    log("smoother %d (matrix_free=%d): oracle iters %s gpu %s err %.3e"
        % (smoother, mf, ores[0]["pcg_iters"].tolist(), gres[0]["pcg_iters"].tolist(), err))
    assert (gres[0]["pcg_ratio"] <= 1e-6).all()
    for a, b in zip(ores[0]["pcg_iters"], gres[0]["pcg_iters"]):
        assert iters_close(a, b)
    assert err <= 1e-9


@pytest.mark.parametrize("smoother", [1, 2])
def test_other_smoothers_mixed_and_batched(smoother):
    """FP32 V-cycle with the Chebyshev or Gauss-Seidel smoother, on a batch of
    bodies with their own coefficients and colourings, against the FP64
    oracle."""
    ws = [W.tiny_beam(12, 4, 4, volumes=True, alpha_edge=1e-8, alpha_vol=1e-8, seed=31),
          W.tiny_beam(3, 1, 1, seed=32),
          W.perturbed(W.tiny_beam(20, 3, 3, volumes=True, alpha_edge=1e-7, alpha_vol=1e-8,
                                  seed=33), 1e-3)]
    oo, _ = opts(smoother=smoother, coarse_max=60)
    for prec, bound in ((B.PREC_FP64, 1e-9), (B.PREC_MIXED, 1e-7)):
        _, go = opts(smoother=smoother, coarse_max=60, precision=prec)
        batch = B.Batch(ws, go)
        res = batch.step(5)
        for k, w in enumerate(ws):
            sim = O.Sim(w, oo)
            pos, vel = O.positions(w)
            sim.step(pos, vel, 5)
            err = rel_pos_err(batch.bodies[k].positions(), pos)
            log("smoother %d batch precision %d body %d: iters %s err %.3e"
                % (smoother, prec, k, res[k]["pcg_iters"].tolist(), err))
            assert (res[k]["pcg_ratio"] <= 1e-6).all()
            assert err <= bound
        batch.close()


@pytest.mark.parametrize("mf,arap", [(1, False), (0, False), (1, True)])
def test_apply_entry_matches_assembled_matrix(mf, arap):
    """mgpbd_apply (the PCG loop's own fine-level product) against the
    assembled A of the same iteration, multiplied on the host: equal up to
    the order of the sums (1e-13 of |A| |x| per row)."""
    import scipy.sparse as sp
    w = W.arap_beam(12, 4, 4, seed=61, squash=0.1) if arap else W.beam_c0()
    _, go = opts(matrix_free=mf, lmax_scale=1.5 if arap else 1.05)
    body = B.Body(w, go)
    body.step(1)
    rp, col, val = B.mgpbd_get_matrix(body.ctx, 0)
    A = sp.csr_matrix((val, col, rp))
    m = rp.size - 1
    x = np.random.default_rng(3).standard_normal(m)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    yt = torch.empty_like(xt)
    B.mgpbd_apply(body.ctx, xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    ref = A @ x
    scale = abs(A) @ np.abs(x)
    err = float((np.abs(y - ref) / scale).max())
    log("apply (matrix_free=%d, arap=%s): max row error %.3e of |A||x|" % (mf, arap, err))
    body.close()
    assert err <= 1e-13
    solver = B.mgpbd_solver_create(go)   # no assembled system: E_STATE
    with pytest.raises(B.MgpbdError):
        B.mgpbd_apply(solver, xt, yt)
    B.mgpbd_destroy(solver)


def test_solve_entry_mixed_precision_reaches_tolerance():
    """mgpbd_solve with the FP32 V-cycle (flexible PCG): the same aggregates
    as the FP64 oracle's setup and an FP64 true residual at the tolerance."""
    import scipy.sparse as sp
    w = W.perturbed(W.tiny_beam(12, 4, 4, volumes=True, alpha_edge=1e-8, alpha_vol=1e-8), 0.01)
    sim = O.Sim(w)
    val, b = sim.assemble(w.x0)
    rp, col = sim.pattern()
    oo, go = opts(coarse_max=60, precision=B.PREC_MIXED)
    h = O.Hier.build(rp, col, val, oo)
    ctx = B.mgpbd_solver_create(go)
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    xg = torch.zeros(sim.m, dtype=torch.float64, device="cuda")
    r = B.mgpbd_solve(ctx, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.float64),
                      dev(b, torch.float64), 1e-8, xg)
    assert r["status"] == B.OK
    for l in range(h.levels - 1):
        assert np.array_equal(B.mgpbd_get_aggregates(ctx, l), h.transfer(l)[0])
    x = xg.cpu().numpy()
    A = sp.csr_matrix((val, col, rp))
    rel = float(np.linalg.norm(A @ x - b) / np.linalg.norm(b))
    log("mixed solve: %d iterations, true residual %.3e" % (r["iters"], rel))
    assert rel <= 1.5e-8
    B.mgpbd_destroy(ctx)


def test_body_without_constraints_is_a_plain_euler_step():
    """No constraint rows: every global iteration is empty and the frame is
    the semi-implicit Euler step of Algorithm 1 alone, as in the oracle."""
    w = W.tiny_beam(2, 1, 1)
    w.edges = np.zeros((0, 2), np.int32)
    w.vol_tet = np.zeros(0, np.int32)
    w.alpha = np.zeros(0)
    oo, go = opts()
    sim = O.Sim(w, oo)
    pos, vel = O.positions(w)
    r = sim.step(pos, vel, 3)
    assert r["status"] == 0
    body = B.Body(w, go)
    assert body.m == 0
    for _ in range(2):
        body.step(3)
    sim.step(pos, vel, 3)
    assert np.array_equal(body.positions(), pos)
    assert np.array_equal(body.velocities(), vel)
    body.close()


def test_frame_with_zero_iterations_then_lazy_frames():
    """n_iters = 0: the frame is the predict and velocity steps of Algorithm 1
    alone (bit-exact with the oracle) and counts as a frame; the next frames
    set up lazily on the same schedule as the oracle and match it. Each later
    frame starts the GPU body from the oracle's positions and velocities (the
    hierarchy and the schedule still carry over): chained frames of this beam
    amplify rounding-level differences past 1e-9 (the oracle against itself
    with omega changed by 1e-14 relative differs by 5e-10 after two such
    frames), so the 1e-9 bar applies per frame."""
    w = W.beam_c0()
    oo, go = opts()
    sim = O.Sim(w, oo)
    pos, vel = O.positions(w)
    body = B.Body(w, go)
    ro = sim.step(pos, vel, 0)
    rg = body.step(0)
    assert ro["status"] == 0 and rg["iters_done"] == 0
    assert np.array_equal(body.positions(), pos)
    assert np.array_equal(body.velocities(), vel)
    for f in range(2):
        for k in range(3):
            body.x[k].copy_(torch.from_numpy(np.ascontiguousarray(pos[:, k])))
            body.v[k].copy_(torch.from_numpy(np.ascontiguousarray(vel[:, k])))
        ro = sim.step(pos, vel, 4)
        assert ro["status"] == 0
        B.mgpbd_force_pcg_iters(body.ctx, ro["pcg_iters"])
        rg = body.step(4)
        assert (rg["setup_ran"] == ro["setup"]).all(), (rg["setup_ran"], ro["setup"])
        err = rel_pos_err(body.positions(), pos)
        log("frame %d after an empty frame: setup %s position err %.3e"
            % (f + 1, rg["setup_ran"].tolist(), err))
        assert err <= 1e-9
    body.close()


def test_fully_pinned_bodies():
    """Every vertex pinned (inverse mass 0): with compliant rows A is the
    diagonal of compliances, b = 0 and nothing moves, as in the oracle (bit
    for bit); with rigid rows (compliance 0) A is the zero matrix and both
    sides report the same breakdown status."""
    w = W.tiny_beam(3, 1, 1)
    w.inv_mass = np.zeros_like(w.inv_mass)
    oo, go = opts()
    sim = O.Sim(w, oo)
    pos, vel = O.positions(w)
    ro = sim.step(pos, vel, 2)
    assert ro["status"] == 0
    body = B.Body(w, go)
    rg = body.step(2)
    assert np.array_equal(body.positions(), pos)
    assert np.array_equal(body.velocities(), vel)
    assert (rg["pcg_iters"] == 0).all() and (rg["bnorm"] == 0).all()
    rp, col, val = B.mgpbd_get_matrix(body.ctx, 0)
    body.close()
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    assert (val[rows != col] == 0).all()
    assert (val[rows == col] > 0).all()
    w.alpha = np.zeros_like(w.alpha)
    sim = O.Sim(w, oo)
    pos, vel = O.positions(w)
    ro = sim.step(pos, vel, 2)
    assert ro["status"] == B.E_BREAKDOWN
    body = B.Body(w, go)
    with pytest.raises(B.MgpbdError) as e:
        body.step(2)
    log("rigid fully pinned body: oracle status %d, library %s" % (ro["status"], e.value))
    assert e.value.status == B.E_BREAKDOWN
    body.close()


@pytest.mark.gpu
def test_failed_frame_leaves_positions_and_velocities_unchanged():
    """A frame that fails inside Algorithm 1's loop (here the setup meets a
    zero diagonal: a rigid edge between two pinned vertices, which the oracle
    also reports as a breakdown) hands the caller back the positions and
    velocities it passed in, bit for bit, although the predict had already
    moved the free vertices; the same holds for a batch."""
    w = W.tiny_beam(3, 1, 1)
    pinned = w.inv_mass == 0
    rigid = pinned[w.edges[:, 0]] & pinned[w.edges[:, 1]]
    assert rigid.any() and not pinned.all()
    w.alpha = np.where(np.concatenate([rigid, np.zeros(w.vol_tet.shape[0], bool)]), 0.0, w.alpha)
    w.v0 = np.where(pinned[:, None], 0.0,
                    np.random.default_rng(3).uniform(-0.1, 0.1, w.v0.shape))
    oo, go = opts()
    pos, vel = O.positions(w)
    assert O.Sim(w, oo).step(pos, vel, 2)["status"] == B.E_BREAKDOWN
    body = B.Body(w, go)
    x0, v0 = body.positions(), body.velocities()
    with pytest.raises(B.MgpbdError) as e:
        body.step(2)
    assert e.value.status == B.E_BREAKDOWN
    assert np.array_equal(body.positions(), x0) and np.array_equal(body.velocities(), v0)
    assert np.array_equal(x0, w.x0) and np.array_equal(v0, w.v0)
    body.close()
    good = W.tiny_beam(4, 1, 1)
    batch = B.Batch([good, w], go)
    xs = [b.positions() for b in batch.bodies]
    vs = [b.velocities() for b in batch.bodies]
    with pytest.raises(B.MgpbdError) as e:
        batch.step(2)
    assert e.value.status == B.E_BREAKDOWN
    for b, x, v in zip(batch.bodies, xs, vs):
        assert np.array_equal(b.positions(), x) and np.array_equal(b.velocities(), v)
    batch.close()


@pytest.mark.parametrize("fuse,mf,smoother", [(1, 1, 0), (0, 1, 0), (1, 0, 0), (0, 0, 0),
                                              (1, 1, 1), (1, 0, 1)])
def test_transfer_forms_match_oracle(fuse, mf, smoother):
    """Residual + restriction in one pass and the prolongation folded into the
    first post-sweep (fuse 1) or separate kernels (fuse 0, the default), with
    matrix-free or assembled fine levels, Jacobi or Chebyshev smoothing: a
    three-level hierarchy against the oracle at forced PCG counts."""
    w = W.beam(48, 12, 12, seed=5, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9)
    sim, body, pos, vel, ores, gres = run_both(w, 3, force_from_oracle=True, coarse_max=100,
                                               fuse_transfers=fuse, matrix_free=mf,
                                               smoother=smoother)
    levels = [B.mgpbd_get_level(body.ctx, l)["n"] for l in range(B.mgpbd_num_levels(body.ctx))]
    err = rel_pos_err(body.positions(), pos)
    log("fuse %d mf %d smoother %d: levels %s, position error %.3e" % (fuse, mf, smoother, levels,
                                                                     err))
    assert len(levels) >= 3
    assert err <= 1e-9
