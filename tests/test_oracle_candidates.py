"""Pins of the oracle's K-candidate setup (Sec. 4.3 generates six near-kernel
vectors; Sec. 4.1 forms each next level from a QR factorisation of them):
per aggregate a modified Gram-Schmidt QR with dependent columns dropped, P
from the Q factors, the next level's candidates from the R factors. Checked
against dense linear algebra (numpy), not against the oracle itself.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_pins import dense, small_hier


def dense_p(h, l, K):
    """Dense P of level l from the aggregates and the stored Q blocks."""
    info = h.info(l)
    agg, _, _ = h.transfer(l)
    kq, coff, Q, B = h.transfer_qr(l, K)
    n = info["n"]
    P = np.zeros((n, int(coff[-1])))
    # member slots in the order of the ascending aggregate lists
    slot = 0
    for a in range(info["n_agg"]):
        for i in np.nonzero(agg == a)[0]:
            P[i, coff[a]:coff[a] + kq[a]] = Q[slot, :kq[a]]
            assert not Q[slot, kq[a]:].any()
            slot += 1
    return P, agg, kq, coff, B


@pytest.mark.parametrize("K", [2, 6])
def test_block_qr_prolongator_and_galerkin(K):
    """P^T P = I; every kept column comes from the candidates (P R = B on
    the aggregated rows, up to the dropped parts); coarse matrix = dense
    P^T A P, symmetric positive definite; 1 <= kq <= min(K, aggregate size)."""
    w, s, rp, col, val, b, h = small_hier(n_cand=K)
    assert h.levels >= 2
    for l in range(h.levels - 1):
        rpl, coll, vall = h.matrix(l)
        P, agg, kq, coff, B = dense_p(h, l, K)
        sizes = np.bincount(agg[agg >= 0], minlength=kq.size)
        assert (kq >= 1).all() and (kq <= np.minimum(K, sizes)).all()
        nc = P.shape[1]
        assert np.allclose(P.T @ P, np.eye(nc), atol=1e-13)
        rpc, colc, valc = h.matrix(l + 1)
        Ac = dense(rpc, colc, valc, nc)
        ref = P.T @ dense(rpl, coll, vall) @ P
        assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.array_equal(Ac, Ac.T)
        assert np.linalg.eigvalsh(Ac).min() > 0
        # the next level's candidates reproduce this level's: P B_{l+1} = B_l
        # (columns dropped as dependent leave at most 1e-8 of their norm)
        _, _, _, Bn = h.transfer_qr(l + 1, K) if l + 1 < h.levels - 1 else (0, 0, 0, None)
        if Bn is None:
            # last level: rebuild B_{l+1} as P^T B_l (what R holds)
            Bn = P.T @ B
        idx = agg >= 0
        err = np.abs(P @ Bn - B)[idx].max()
        assert err <= 2e-8 * np.abs(B[idx]).max()


def test_identical_candidates_keep_one_column():
    """With all candidates equal (the all-ones mode) every aggregate keeps one
    column and the hierarchy equals the one-candidate hierarchy bit for bit."""
    _, _, _, _, _, _, h1 = small_hier(b_mode=1)
    _, _, _, _, _, _, h6 = small_hier(b_mode=1, n_cand=6)
    assert h1.levels == h6.levels
    for l in range(h1.levels):
        for u, v in zip(h1.matrix(l), h6.matrix(l)):
            assert np.array_equal(u, v)
        if l + 1 < h1.levels:
            kq, _, _, _ = h6.transfer_qr(l, 6)
            assert (kq == 1).all()
            a1, p1, _ = h1.transfer(l)
            a6, p6, _ = h6.transfer(l)
            assert np.array_equal(a1, a6) and np.array_equal(p1, p6)


def test_mgpcg_with_six_candidates_matches_dense_solve():
    w, s, rp, col, val, b, h = small_hier(n_cand=6)
    x, st = h.pcg(b, 1e-10, 2000)
    A = dense(rp, col, val)
    assert st["status"] == 0
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
    rng = np.random.default_rng(5)
    for _ in range(4):
        y, z = rng.standard_normal((2, s.m))
        a1, a2 = z @ h.vcycle(y), y @ h.vcycle(z)
        assert abs(a1 - a2) <= 1e-13 * (abs(a1) + abs(a2))
        assert y @ h.vcycle(y) > 0


def test_candidate_option_range():
    _, s, rp, col, val, _, _ = small_hier()
    with pytest.raises(O.OracleError):
        O.Hier.build(rp, col, val, O.default_opts(n_cand=0))
    with pytest.raises(O.OracleError):
        O.Hier.build(rp, col, val, O.default_opts(n_cand=9))
