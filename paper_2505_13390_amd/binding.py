"""Thin ctypes binding of the C ABI in include/mgpbd.h.

Argument marshalling only: every step runs in the HIP library. Device
arrays are torch cuda tensors (float64 / int32 / int64, contiguous); their
data pointers are handed to the library together with the current torch
stream. The library must be built (paper_2505_13390_amd/build.py); there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgpbd_hip.so")

OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_DEVICE, E_NOT_CONVERGED, E_BREAKDOWN, E_SETUP, E_STATE = range(8)
PREC_FP64, PREC_MIXED = 0, 1


class Options(C.Structure):
    _fields_ = [("theta", C.c_double), ("gs_sweeps", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_sweeps", C.c_int32), ("lambda_min", C.c_double),
                ("coarse_max", C.c_int32), ("dense_max", C.c_int32), ("max_levels", C.c_int32),
                ("power_iters", C.c_int32), ("omega_relax", C.c_double), ("tol", C.c_double),
                ("max_pcg", C.c_int32), ("seed", C.c_uint64), ("reuse_interval", C.c_int32),
                ("b_mode", C.c_int32), ("eps_b", C.c_double), ("precision", C.c_int32),
                ("lmax_scale", C.c_double), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("profile_spmv", C.c_int32),
                ("spmv_tile", C.c_int32), ("spmv_lanes", C.c_int32),
                ("matrix_free", C.c_int32), ("smoother", C.c_int32), ("n_cand", C.c_int32),
                ("power_max", C.c_int32), ("power_tol", C.c_double),
                ("vcycle_tail", C.c_int32), ("fuse_transfers", C.c_int32),
                ("resetup_on_breakdown", C.c_int32)]


class Mesh(C.Structure):
    _fields_ = [("n_verts", C.c_int64), ("rest", C.c_void_p), ("inv_mass", C.c_void_p),
                ("n_tets", C.c_int64), ("tets", C.c_void_p)]


class Constraints(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("edges", C.c_void_p), ("n_vols", C.c_int64),
                ("vol_tet", C.c_void_p), ("n_arap", C.c_int64), ("arap_tet", C.c_void_p)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class StepStats(C.Structure):
    _fields_ = [("bnorm", C.c_void_p), ("pcg_iters", C.c_void_p), ("pcg_ratio", C.c_void_p),
                ("setup_ran", C.c_void_p), ("iters_done", C.c_int32), ("ms_setup", C.c_double),
                ("ms_pcg", C.c_double), ("ms_total", C.c_double), ("spmv_calls", C.c_int64),
                ("spmv_ms", C.c_double), ("spmv_first_ms", C.c_double),
                ("ms_assembly", C.c_double), ("ms_galerkin", C.c_double),
                ("ms_update", C.c_double), ("vcycles", C.c_int64),
                ("ms_level", C.c_double * 16)]


def _phase_fields(st, levels):
    """The per-phase timers of a filled StepStats (levels: how many of
    ms_level to report)."""
    return dict(ms_assembly=st.ms_assembly, ms_galerkin=st.ms_galerkin, ms_update=st.ms_update,
                vcycles=st.vcycles, ms_level=[st.ms_level[l] for l in range(levels)])


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ratio", C.c_double), ("ms_setup", C.c_double),
                ("ms_solve", C.c_double)]


class MgpbdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("mgpbd status %d: %s" % (status, msg))
        self.status = status


_lib = None

_SIGS = {
    "mgpbd_default_options": (None, [C.POINTER(Options)]),
    "mgpbd_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Constraints), C.c_void_p, C.c_double,
                               C.c_void_p, C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "mgpbd_solver_create": (C.c_int, [C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "mgpbd_setup": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "mgpbd_step": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6 + [C.c_int32, C.POINTER(StepStats)]),
    "mgpbd_solve": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.c_void_p, C.c_double, C.c_void_p,
                              C.POINTER(SolveStats)]),
    "mgpbd_destroy": (None, [C.c_void_p]),
    "mgpbd_last_error": (C.c_char_p, [C.c_void_p]),
    "mgpbd_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgpbd_force_pcg_iters": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "mgpbd_num_rows": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mgpbd_num_levels": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mgpbd_get_level": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_int64)]),
    "mgpbd_get_aggregates": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mgpbd_get_transfer": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mgpbd_get_matrix": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mgpbd_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mgpbd_apply_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mgpbd_get_qr": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "mgpbd_get_fine_operator": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mgpbd_get_rhs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgpbd_get_lambda": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgpbd_get_colors": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "mgpbd_selftest_sqrt_div": (C.c_int, [C.c_int64] + [C.c_void_p] * 4),
    "mgpbd_batch_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "mgpbd_batch_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "mgpbd_batch_context": (C.c_void_p, [C.c_void_p]),
    "mgpbd_batch_destroy": (None, [C.c_void_p]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load the HIP library; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run paper_2505_13390_amd/build.py"
                               % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev(t, dtype=None):
    """Device pointer of a contiguous cuda tensor (checks dtype/device)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a cuda tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _vec(t, dtype, n, what):
    """_dev plus a length check: the library reads and writes exactly n
    entries through the pointer and cannot see the tensor's size."""
    p = _dev(t, dtype)
    if t.numel() != n:
        raise ValueError("%s has %d entries, expected %d" % (what, t.numel(), n))
    return p


# vertex counts of the contexts and batches created here, for the length
# checks of the calls that take per-vertex device arrays
_NV = {}
_BATCH_NV = {}


def _key(h):
    return h.value if isinstance(h, C.c_void_p) else int(h)


def _check(ctx, st):
    if st != OK:
        msg = lib().mgpbd_last_error(ctx) if ctx else b""
        raise MgpbdError(st, (msg or b"").decode())


def mgpbd_default_options(**overrides) -> Options:
    o = Options()
    lib().mgpbd_default_options(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prepare(ctx):
    """Order the library's work after torch's: use torch's current stream; if
    that is the legacy default stream (which the library does not capture
    graphs on), wait for the device first and let the library use its own
    stream. The library itself returns only after its work has completed."""
    import torch
    s = torch.cuda.current_stream().cuda_stream
    _check(ctx, lib().mgpbd_set_stream(ctx, C.c_void_p(s) if s else None))
    if not s:
        torch.cuda.synchronize()


def mgpbd_create(rest, inv_mass, tets, edges, vol_tet, compliance, dt, gravity,
                 opt: Options | None = None, arap_tet=None):
    """Create a body context from host arrays (numpy). Returns the handle.
    Rows: edges, then volume rows (vol_tet), then ARAP rows (arap_tet)."""
    rest = np.ascontiguousarray(rest, np.float64)
    inv_mass = np.ascontiguousarray(inv_mass, np.float64)
    tets = np.ascontiguousarray(tets, np.int32).reshape(-1, 4)
    edges = np.ascontiguousarray(edges, np.int32).reshape(-1, 2)
    vol_tet = np.ascontiguousarray(vol_tet, np.int32)
    arap_tet = np.ascontiguousarray(np.zeros(0) if arap_tet is None else arap_tet, np.int32)
    comp = np.ascontiguousarray(compliance, np.float64)
    grav = np.ascontiguousarray(gravity, np.float64)
    mesh = Mesh(rest.shape[0], _np_ptr(rest).value, _np_ptr(inv_mass).value, tets.shape[0],
                _np_ptr(tets).value)
    cons = Constraints(edges.shape[0], _np_ptr(edges).value, vol_tet.shape[0],
                       _np_ptr(vol_tet).value, arap_tet.shape[0], _np_ptr(arap_tet).value)
    h = C.c_void_p()
    st = lib().mgpbd_create(C.byref(mesh), C.byref(cons), _np_ptr(comp), float(dt),
                            _np_ptr(grav), C.byref(opt) if opt is not None else None, C.byref(h))
    if st != OK:
        raise MgpbdError(st, "mgpbd_create")
    _NV[_key(h)] = rest.shape[0]
    return h


def mgpbd_solver_create(opt: Options | None = None):
    h = C.c_void_p()
    st = lib().mgpbd_solver_create(C.byref(opt) if opt is not None else None, C.byref(h))
    if st != OK:
        raise MgpbdError(st, "mgpbd_solver_create")
    return h


def mgpbd_setup(ctx, max_levels: int, reuse_interval: int):
    _check(ctx, lib().mgpbd_setup(ctx, max_levels, reuse_interval))


def mgpbd_step(ctx, x, y, z, vx, vy, vz, n_iters: int, stats: bool = True):
    import torch
    f64 = torch.float64
    nv = _NV.get(_key(ctx), x.numel())
    for t, what in zip((x, y, z, vx, vy, vz), ("x", "y", "z", "vx", "vy", "vz")):
        _vec(t, f64, nv, what)
    n = max(int(n_iters), 1)
    bn = np.zeros(n)
    its = np.zeros(n, np.int32)
    ratio = np.zeros(n)
    setup = np.zeros(n, np.int32)
    st = StepStats(_np_ptr(bn).value, _np_ptr(its).value, _np_ptr(ratio).value,
                   _np_ptr(setup).value)
    _prepare(ctx)
    s = lib().mgpbd_step(ctx, _dev(x, f64), _dev(y, f64), _dev(z, f64), _dev(vx, f64),
                         _dev(vy, f64), _dev(vz, f64), int(n_iters),
                         C.byref(st) if stats else None)
    _check(ctx, s)
    k = st.iters_done
    return dict(bnorm=bn[:k], pcg_iters=its[:k], pcg_ratio=ratio[:k], setup_ran=setup[:k],
                iters_done=k, ms_setup=st.ms_setup, ms_pcg=st.ms_pcg, ms_total=st.ms_total,
                spmv_calls=st.spmv_calls, spmv_ms=st.spmv_ms, spmv_first_ms=st.spmv_first_ms,
                **_phase_fields(st, 16))


def mgpbd_solve(ctx, rowptr, col, val, b, tol, x_out):
    import torch
    n = rowptr.numel() - 1
    if n < 0:
        raise ValueError("rowptr must hold n + 1 entries")
    _vec(val, torch.float64, col.numel(), "val")
    _vec(b, torch.float64, n, "b")
    _vec(x_out, torch.float64, n, "x_out")
    csr = Csr(rowptr.numel() - 1, col.numel(), _dev(rowptr, torch.int64).value,
              _dev(col, torch.int32).value, _dev(val, torch.float64).value)
    st = SolveStats()
    _prepare(ctx)
    s = lib().mgpbd_solve(ctx, C.byref(csr), _dev(b, torch.float64), float(tol),
                          _dev(x_out, torch.float64), C.byref(st))
    if s not in (OK, E_NOT_CONVERGED):
        _check(ctx, s)
    return dict(status=s, iters=st.iters, ratio=st.ratio, ms_setup=st.ms_setup,
                ms_solve=st.ms_solve)


def mgpbd_destroy(ctx):
    if ctx:
        _NV.pop(_key(ctx), None)
        lib().mgpbd_destroy(ctx)


def mgpbd_set_stream(ctx, stream_ptr: int):
    _check(ctx, lib().mgpbd_set_stream(ctx, C.c_void_p(stream_ptr)))


def mgpbd_force_pcg_iters(ctx, iters):
    if iters is None:
        _check(ctx, lib().mgpbd_force_pcg_iters(ctx, None, 0))
        return
    a = np.ascontiguousarray(iters, np.int32)
    _check(ctx, lib().mgpbd_force_pcg_iters(ctx, _np_ptr(a), a.shape[0]))


def mgpbd_num_rows(ctx):
    m, nnz = C.c_int64(), C.c_int64()
    _check(ctx, lib().mgpbd_num_rows(ctx, C.byref(m), C.byref(nnz)))
    return m.value, nnz.value


def mgpbd_num_levels(ctx):
    l = C.c_int32()
    _check(ctx, lib().mgpbd_num_levels(ctx, C.byref(l)))
    return l.value


def mgpbd_get_level(ctx, l):
    n, nnz, na = C.c_int64(), C.c_int64(), C.c_int64()
    om = C.c_double()
    _check(ctx, lib().mgpbd_get_level(ctx, l, C.byref(n), C.byref(nnz), C.byref(om),
                                      C.byref(na)))
    return dict(n=n.value, nnz=nnz.value, omega=om.value, n_agg=na.value)


def mgpbd_get_aggregates(ctx, l):
    n = mgpbd_get_level(ctx, l)["n"]
    out = np.zeros(n, np.int32)
    _check(ctx, lib().mgpbd_get_aggregates(ctx, l, _np_ptr(out)))
    return out


def mgpbd_get_transfer(ctx, l):
    n = mgpbd_get_level(ctx, l)["n"]
    p = np.zeros(n)
    B = np.zeros(n)
    _check(ctx, lib().mgpbd_get_transfer(ctx, l, _np_ptr(p), _np_ptr(B)))
    return p, B


def mgpbd_get_matrix(ctx, l):
    info = mgpbd_get_level(ctx, l)
    rp = np.zeros(info["n"] + 1, np.int64)
    col = np.zeros(info["nnz"], np.int32)
    val = np.zeros(info["nnz"])
    _check(ctx, lib().mgpbd_get_matrix(ctx, l, _np_ptr(rp), _np_ptr(col), _np_ptr(val)))
    return rp, col, val


def mgpbd_apply(ctx, x, y):
    """y = A x (device FP64 tensors of the context's row count), enqueued on
    the context's stream."""
    import torch
    m, _ = mgpbd_num_rows(ctx)
    if m > 0:   # with no rows the library touches neither array (or reports E_STATE)
        px = _vec(x, torch.float64, m, "x")
        py = _vec(y, torch.float64, m, "y")
    else:
        px, py = _dev(x, torch.float64), _dev(y, torch.float64)
    _check(ctx, lib().mgpbd_apply(ctx, px, py))


def mgpbd_apply_noalloc(ctx, x, y):
    """mgpbd_apply through the entry point that allocates nothing (its gather
    vector lives in the library's static per-GPU scratch array)."""
    import torch
    m, _ = mgpbd_num_rows(ctx)
    if m > 0:
        px = _vec(x, torch.float64, m, "x")
        py = _vec(y, torch.float64, m, "y")
    else:
        px, py = _dev(x, torch.float64), _dev(y, torch.float64)
    _check(ctx, lib().mgpbd_apply_noalloc(ctx, px, py))


def mgpbd_get_qr(ctx, l, n, n_agg, n_mem, K):
    """kq [n_agg], coff [n_agg + 1], Q [n_mem, K], B [n, K] of level l (K > 1)."""
    kq = np.zeros(n_agg, np.int32)
    coff = np.zeros(n_agg + 1, np.int64)
    Q = np.zeros((n_mem, K))
    B = np.zeros((n, K))
    _check(ctx, lib().mgpbd_get_qr(ctx, l, _np_ptr(kq), _np_ptr(coff), _np_ptr(Q), _np_ptr(B)))
    return kq, coff, Q, B


def mgpbd_get_fine_operator(ctx):
    """1 when the fine-level passes are matrix-free, 0 when assembled"""
    v = C.c_int32(0)
    _check(ctx, lib().mgpbd_get_fine_operator(ctx, C.byref(v)))
    return int(v.value)


def mgpbd_get_rhs(ctx, m):
    out = np.zeros(m)
    _check(ctx, lib().mgpbd_get_rhs(ctx, _np_ptr(out)))
    return out


def mgpbd_get_lambda(ctx, m):
    out = np.zeros(m)
    _check(ctx, lib().mgpbd_get_lambda(ctx, _np_ptr(out)))
    return out


def mgpbd_get_colors(ctx, m):
    out = np.zeros(m, np.int32)
    nc = C.c_int32()
    _check(ctx, lib().mgpbd_get_colors(ctx, _np_ptr(out), C.byref(nc)))
    return out, nc.value


def mgpbd_selftest_sqrt_div(a, b):
    import torch
    _vec(b, torch.float64, a.numel(), "b")
    s = torch.empty_like(a)
    q = torch.empty_like(a)
    torch.cuda.synchronize()
    st = lib().mgpbd_selftest_sqrt_div(a.numel(), _dev(a, torch.float64), _dev(b, torch.float64),
                                       _dev(s, torch.float64), _dev(q, torch.float64))
    if st != OK:
        raise MgpbdError(st, "selftest")
    return s, q


def mgpbd_batch_create(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    h = C.c_void_p()
    st = lib().mgpbd_batch_create(arr, len(ctxs), C.byref(h))
    if st != OK:
        msg = lib().mgpbd_last_error(arr[0]) if len(ctxs) and arr[0] else b""
        raise MgpbdError(st, "mgpbd_batch_create: " + (msg or b"").decode())
    _BATCH_NV[_key(h)] = [_NV.get(_key(c)) for c in ctxs]
    return h


def mgpbd_batch_context(batch):
    return C.c_void_p(lib().mgpbd_batch_context(batch))


def mgpbd_batch_step(batch, xyz_list, vxyz_list, n_iters, stats: bool = True):
    """One frame for every body of the batch; returns one stats dict per body."""
    import torch
    nb = len(xyz_list)
    sizes = _BATCH_NV.get(_key(batch))
    if len(vxyz_list) != nb or (sizes is not None and len(sizes) != nb):
        raise ValueError("expected positions and velocities for every body of the batch")
    xs = (C.c_void_p * (3 * nb))()
    vs = (C.c_void_p * (3 * nb))()
    for k, (p, v) in enumerate(zip(xyz_list, vxyz_list)):
        nv = sizes[k] if sizes is not None and sizes[k] is not None else p[0].numel()
        for d in range(3):
            xs[3 * k + d] = _vec(p[d], torch.float64, nv, "body %d position" % k).value
            vs[3 * k + d] = _vec(v[d], torch.float64, nv, "body %d velocity" % k).value
    n = max(int(n_iters), 1)
    arrs = [dict(bnorm=np.zeros(n), pcg_iters=np.zeros(n, np.int32), pcg_ratio=np.zeros(n),
                 setup_ran=np.zeros(n, np.int32)) for _ in range(nb)]
    sts = (StepStats * nb)()
    for k, a in enumerate(arrs):
        sts[k] = StepStats(_np_ptr(a["bnorm"]).value, _np_ptr(a["pcg_iters"]).value,
                           _np_ptr(a["pcg_ratio"]).value, _np_ptr(a["setup_ran"]).value)
    sys_ctx = mgpbd_batch_context(batch)
    _prepare(sys_ctx)
    st = lib().mgpbd_batch_step(batch, xs, vs, int(n_iters), sts if stats else None)
    _check(sys_ctx, st)
    out = []
    for k, a in enumerate(arrs):
        d = sts[k].iters_done
        out.append(dict(bnorm=a["bnorm"][:d], pcg_iters=a["pcg_iters"][:d],
                        pcg_ratio=a["pcg_ratio"][:d], setup_ran=a["setup_ran"][:d],
                        iters_done=d, ms_setup=sts[k].ms_setup, ms_pcg=sts[k].ms_pcg,
                        ms_total=sts[k].ms_total, spmv_calls=sts[k].spmv_calls,
                        spmv_ms=sts[k].spmv_ms, spmv_first_ms=sts[k].spmv_first_ms,
                        **_phase_fields(sts[k], 16)))
    return out


def mgpbd_batch_destroy(batch):
    if batch:
        _BATCH_NV.pop(_key(batch), None)
        lib().mgpbd_batch_destroy(batch)


class Body:
    """Convenience owner of one body context and its device state."""

    def __init__(self, w, opt: Options | None = None, device="cuda:0"):
        import torch
        self.w = w
        self.ctx = mgpbd_create(w.rest, w.inv_mass, w.tets, w.edges, w.vol_tet, w.alpha, w.dt,
                                w.gravity, opt, arap_tet=w.arap_tet)
        self.m, self.nnz = mgpbd_num_rows(self.ctx)
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
        self.x = [t(w.x0[:, k]) for k in range(3)]
        self.v = [t(w.v0[:, k]) for k in range(3)]

    def step(self, n_iters, stats=True):
        return mgpbd_step(self.ctx, *self.x, *self.v, n_iters, stats)

    def positions(self):
        return np.stack([a.cpu().numpy() for a in self.x], axis=1)

    def velocities(self):
        return np.stack([a.cpu().numpy() for a in self.v], axis=1)

    def close(self):
        if self.ctx:
            mgpbd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several bodies stepped together as one block-diagonal system."""

    def __init__(self, workloads, opt: Options | None = None, device="cuda:0"):
        self.bodies = [Body(w, opt, device) for w in workloads]
        self.h = mgpbd_batch_create([b.ctx for b in self.bodies])
        self.ctx = mgpbd_batch_context(self.h)

    def step(self, n_iters, stats=True):
        return mgpbd_batch_step(self.h, [b.x for b in self.bodies], [b.v for b in self.bodies],
                                n_iters, stats)

    def close(self):
        if self.h:
            mgpbd_batch_destroy(self.h)
            self.h = None
        for b in self.bodies:
            b.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
