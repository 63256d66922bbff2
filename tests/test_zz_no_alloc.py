"""mgpbd_apply_noalloc, the entry point that allocates nothing, against
mgpbd_apply on the same context and input: two calls in a row through the C
ABI, the second on a smaller body, both bit-identical (same kernels, same
inputs; only where the gather vector lives differs). Also the size limit of
its static scratch array."""
import numpy as np
import pytest

from paper_2505_13390_amd import workloads as W
from tests.gpu_common import B, log, opts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _body(w, **kw):
    _, go = opts(**kw)
    body = B.Body(w, go)
    B.mgpbd_force_pcg_iters(body.ctx, [5])
    body.step(1)
    return body


def _check_pair(body, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(body.m, dtype=torch.float64, generator=g).cuda()
    y_ref = torch.full_like(x, np.nan)
    y = torch.full_like(x, np.nan)
    B.mgpbd_apply(body.ctx, x, y_ref)
    torch.cuda.synchronize()
    B.mgpbd_apply_noalloc(body.ctx, x, y)
    torch.cuda.synchronize()
    a, b = y.cpu().numpy(), y_ref.cpu().numpy()
    nbad = int((a.view(np.uint64) != b.view(np.uint64)).sum())
    log("noalloc vs apply: %d rows, %d verts, %d differ" % (body.m, body.w.n_verts, nbad))
    assert np.isfinite(a).all() and nbad == 0


@pytest.mark.parametrize("matrix_free", [1, 0])
def test_noalloc_matches_apply(matrix_free):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = _body(W.beam(48, 12, 12, seed=5, volumes=True, alpha_edge=1e-8, alpha_vol=1e-9),
                matrix_free=matrix_free)
    small = _body(W.tiny_beam(6, 2, 2, volumes=True), matrix_free=matrix_free)
    assert small.w.n_verts < big.w.n_verts
    _check_pair(big, 1)
    _check_pair(small, 2)
    # and the big one again after the small call left its values in the array
    _check_pair(big, 3)
    big.close()
    small.close()


def test_noalloc_size_limit():
    """A body with more vertices than the scratch array holds is refused
    before anything is enqueued."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = W.beam(168, 48, 64, seed=3, volumes=False, alpha_edge=1e-8)
    assert 32 * w.n_verts > 16 << 20
    body = _body(w)
    x = torch.zeros(body.m, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(B.MgpbdError) as e:
        B.mgpbd_apply_noalloc(body.ctx, x, y)
    assert e.value.status == B.E_INVALID_ARG
    log("size limit:", str(e.value))
    body.close()
