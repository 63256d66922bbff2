"""The binding's argument checks on the GPU: the C ABI takes bare device
pointers and cannot see a tensor's length, so the binding rejects short,
long, non-contiguous, host or wrongly typed tensors before the library runs
(a short output would otherwise be written past its end). Every rejected
call leaves the context usable."""
import numpy as np
import pytest

from paper_2505_13390_amd import binding as B
from paper_2505_13390_amd import workloads as W
from tests.gpu_common import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def test_step_checks_every_state_array():
    w = W.tiny_beam(4, 2, 2)
    body = B.Body(w)
    nv = w.rest.shape[0]
    good = body.x + body.v
    bad_cases = {
        "short x": torch.zeros(nv - 1, dtype=torch.float64, device="cuda"),
        "long vz": torch.zeros(nv + 1, dtype=torch.float64, device="cuda"),
        "float32 y": torch.zeros(nv, dtype=torch.float32, device="cuda"),
        "strided vx": torch.zeros(2 * nv, dtype=torch.float64, device="cuda")[::2],
    }
    slots = {"short x": 0, "float32 y": 1, "strided vx": 3, "long vz": 5}
    for name, t in bad_cases.items():
        args = list(good)
        args[slots[name]] = t
        with pytest.raises((ValueError, TypeError)):
            B.mgpbd_step(body.ctx, *args, 1)
        log("step rejects %s" % name)
    host = list(good)
    host[2] = torch.zeros(nv, dtype=torch.float64)
    with pytest.raises(TypeError):
        B.mgpbd_step(body.ctx, *host, 1)
    r = body.step(2)
    assert r["iters_done"] == 2 and np.isfinite(body.positions()).all()
    body.close()


def test_apply_and_solve_check_lengths():
    w = W.tiny_beam(4, 2, 2)
    body = B.Body(w)
    body.step(1)
    m = body.m
    x = torch.randn(m, dtype=torch.float64, device="cuda")
    for y in (torch.empty(m - 1, dtype=torch.float64, device="cuda"),
              torch.empty(m + 3, dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            B.mgpbd_apply(body.ctx, x, y)
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    B.mgpbd_apply(body.ctx, x, y)
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
    rp, col, val = B.mgpbd_get_matrix(body.ctx, 0)
    body.close()
    ctx = B.mgpbd_solver_create()
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")
    b = torch.ones(m, dtype=torch.float64, device="cuda")
    args = (dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.float64))
    with pytest.raises(ValueError):
        B.mgpbd_solve(ctx, *args, b, 1e-8, torch.zeros(m - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        B.mgpbd_solve(ctx, *args, b[:-1], 1e-8, torch.zeros(m, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        B.mgpbd_solve(ctx, args[0], args[1], args[2][:-1], b, 1e-8,
                      torch.zeros(m, dtype=torch.float64, device="cuda"))
    xo = torch.zeros(m, dtype=torch.float64, device="cuda")
    r = B.mgpbd_solve(ctx, *args, b, 1e-8, xo)
    assert r["status"] == B.OK
    B.mgpbd_destroy(ctx)


def test_batch_step_checks_every_body():
    ws = [W.tiny_beam(4, 2, 2, seed=1), W.tiny_beam(6, 2, 1, seed=2)]
    batch = B.Batch(ws)
    xs = [list(b.x) for b in batch.bodies]
    vs = [list(b.v) for b in batch.bodies]
    xs[1][2] = xs[1][2][:-1]
    with pytest.raises(ValueError):
        B.mgpbd_batch_step(batch.h, xs, vs, 1)
    with pytest.raises(ValueError):
        B.mgpbd_batch_step(batch.h, [b.x for b in batch.bodies][:1], vs[:1], 1)
    r = batch.step(2)
    assert all(k["iters_done"] == 2 for k in r)
    batch.close()
