"""ctypes wrapper of the FP64 CPU oracle (mgpbd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path. The oracle shares
no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgpbd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_mgpbd.so")

OK, E_INVALID, E_NOMEM, E_NOT_CONVERGED, E_BREAKDOWN, E_SETUP = 0, 1, 2, 4, 5, 6


# MGPBD_ORACLE_LIB names another build of the same source to load instead
# (the sanitizer test builds one with -fsanitize=address,undefined)
_OVERRIDE = os.environ.get("MGPBD_ORACLE_LIB")


def build(force: bool = False) -> str:
    """Compile the oracle (gcc, FP64, no contraction, no fast-math)."""
    if _OVERRIDE:
        return _OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


class Opts(C.Structure):
    _fields_ = [("theta", C.c_double), ("gs_sweeps", C.c_int), ("pre_sweeps", C.c_int),
                ("post_sweeps", C.c_int), ("lambda_min", C.c_double), ("coarse_max", C.c_int),
                ("dense_max", C.c_int), ("max_levels", C.c_int), ("power_iters", C.c_int),
                ("omega_relax", C.c_double), ("tol", C.c_double), ("max_pcg", C.c_int),
                ("seed", C.c_uint64), ("reuse_interval", C.c_int), ("b_mode", C.c_int),
                ("eps_b", C.c_double), ("flexible", C.c_int), ("lmax_scale", C.c_double),
                ("smoother", C.c_int), ("n_cand", C.c_int), ("power_max", C.c_int),
                ("power_tol", C.c_double), ("resetup_on_breakdown", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        P = C.c_void_p
        L.orc_default_opts.argtypes = [C.POINTER(Opts)]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_sim_create.restype = P
        L.orc_sim_create.argtypes = [C.c_int64, P, P, C.c_int64, P, C.c_int64, P, C.c_int64, P,
                                     C.c_int64, P,
                                     P, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(Opts), C.POINTER(C.c_int)]
        L.orc_sim_free.argtypes = [P]
        L.orc_closest_rotation.argtypes = [P, P]
        L.orc_arap_eval.restype = C.c_int
        L.orc_arap_eval.argtypes = [P, P, P, P]
        L.orc_sim_rows.restype = C.c_int64
        L.orc_sim_rows.argtypes = [P]
        L.orc_sim_nnz.restype = C.c_int64
        L.orc_sim_nnz.argtypes = [P]
        L.orc_sim_pattern.argtypes = [P, P, P]
        L.orc_sim_constraints.argtypes = [P, P, P, P]
        L.orc_sim_assemble.argtypes = [P, P, P, P, P]
        L.orc_sim_step.restype = C.c_int
        L.orc_sim_step.argtypes = [P, P, P, C.c_int, P, P, P, P, P]
        L.orc_sim_hier.restype = P
        L.orc_sim_hier.argtypes = [P]
        L.orc_sim_get_lambda.argtypes = [P, P]
        L.orc_sim_get_matrix_values.argtypes = [P, P]
        L.orc_sim_set_frame.argtypes = [P, C.c_int64]
        L.orc_sim_get_rhs.argtypes = [P, P]
        L.orc_sim_invalidate.argtypes = [P]
        L.orc_hier_build.restype = P
        L.orc_hier_build.argtypes = [C.c_int64, P, P, P, C.POINTER(Opts), C.POINTER(C.c_int)]
        L.orc_hier_free.argtypes = [P]
        L.orc_hier_refresh.restype = C.c_int
        L.orc_hier_refresh.argtypes = [P, P]
        L.orc_hier_vcycle.argtypes = [P, P, P]
        L.orc_hier_levels.restype = C.c_int
        L.orc_hier_levels.argtypes = [P]
        L.orc_hier_last_dense.restype = C.c_int
        L.orc_hier_last_dense.argtypes = [P]
        L.orc_hier_level_info.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_hier_level_matrix.argtypes = [P, C.c_int, P, P, P]
        L.orc_hier_level_transfer.restype = C.c_int
        L.orc_hier_level_transfer.argtypes = [P, C.c_int, P, P, P]
        L.orc_hier_level_qr.restype = C.c_int
        L.orc_hier_level_qr.argtypes = [P, C.c_int, P, P, P, P]
        L.orc_hier_coarse_solve.restype = C.c_int
        L.orc_hier_coarse_solve.argtypes = [P, P, P]
        L.orc_hier_colors.restype = C.c_int
        L.orc_hier_colors.argtypes = [P, P]
        L.orc_pcg.restype = C.c_int
        L.orc_pcg.argtypes = [P, P, C.c_double, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_aggregate.restype = C.c_int64
        L.orc_aggregate.argtypes = [C.c_int64, P, P, P, C.c_double, P, P, P]
        L.orc_color.restype = C.c_int
        L.orc_color.argtypes = [C.c_int64, P, P, P, P]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def splitmix64(z: int) -> int:
    return int(lib().orc_splitmix64(z))


def mix64(seed: int, stream: int, i: int) -> int:
    return int(lib().orc_mix64(seed, stream, i))


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed with status %d" % (what, status))
        self.status = status


class Hier:
    """A setup hierarchy (owned or borrowed from a Sim)."""

    def __init__(self, handle, owned: bool):
        self.h = handle
        self.owned = owned

    @classmethod
    def build(cls, rowptr, col, val, opts: Opts | None = None) -> "Hier":
        rowptr = np.ascontiguousarray(rowptr, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        val = np.ascontiguousarray(val, np.float64)
        st = C.c_int(0)
        o = opts if opts is not None else default_opts()
        h = lib().orc_hier_build(rowptr.shape[0] - 1, _p(rowptr), _p(col), _p(val),
                                 C.byref(o), C.byref(st))
        if not h:
            raise OracleError(st.value, "orc_hier_build")
        return cls(h, True)

    def __del__(self):
        if getattr(self, "owned", False) and self.h:
            lib().orc_hier_free(self.h)
            self.h = None

    @property
    def levels(self) -> int:
        return lib().orc_hier_levels(self.h)

    @property
    def last_dense(self) -> bool:
        return bool(lib().orc_hier_last_dense(self.h))

    def info(self, l):
        n, nnz, na = C.c_int64(), C.c_int64(), C.c_int64()
        om, nc = C.c_double(), C.c_int()
        lib().orc_hier_level_info(self.h, l, C.byref(n), C.byref(nnz), C.byref(om),
                                  C.byref(na), C.byref(nc))
        return dict(n=n.value, nnz=nnz.value, omega=om.value, n_agg=na.value, n_colors=nc.value)

    def matrix(self, l):
        i = self.info(l)
        rp = np.zeros(i["n"] + 1, np.int64)
        col = np.zeros(i["nnz"], np.int32)
        val = np.zeros(i["nnz"], np.float64)
        lib().orc_hier_level_matrix(self.h, l, _p(rp), _p(col), _p(val))
        return rp, col, val

    def transfer(self, l):
        n = self.info(l)["n"]
        agg = np.zeros(n, np.int32)
        p = np.zeros(n)
        B = np.zeros(n)
        st = lib().orc_hier_level_transfer(self.h, l, _p(agg), _p(p), _p(B))
        if st != OK:
            raise OracleError(st, "transfer")
        return agg, p, B

    def transfer_qr(self, l, K):
        """kq [n_agg], coff [n_agg + 1], Q [members, K], B [n, K] of level l."""
        info = self.info(l)
        n, na = info["n"], info["n_agg"]
        kq = np.zeros(na, np.int32)
        coff = np.zeros(na + 1, np.int64)
        agg, _, _ = self.transfer(l)
        nmem = int((agg >= 0).sum())
        Q = np.zeros((nmem, K))
        B = np.zeros((n, K))
        st = lib().orc_hier_level_qr(self.h, l, _p(kq), _p(coff), _p(Q), _p(B))
        if st != OK:
            raise OracleError(st, "transfer_qr")
        return kq, coff, Q, B

    def colors(self):
        n = self.info(0)["n"]
        c = np.zeros(n, np.int32)
        nc = lib().orc_hier_colors(self.h, _p(c))
        return c, nc

    def refresh(self, val0):
        val0 = np.ascontiguousarray(val0, np.float64)
        st = lib().orc_hier_refresh(self.h, _p(val0))
        if st != OK:
            raise OracleError(st, "refresh")

    def coarse_solve(self, r):
        """z = A_L^-1 r with the last level's dense factor."""
        r = np.ascontiguousarray(r, np.float64)
        z = np.zeros_like(r)
        st = lib().orc_hier_coarse_solve(self.h, _p(r), _p(z))
        if st != OK:
            raise OracleError(st, "coarse_solve")
        return z

    def vcycle(self, r):
        r = np.ascontiguousarray(r, np.float64)
        z = np.zeros_like(r)
        lib().orc_hier_vcycle(self.h, _p(r), _p(z))
        return z

    def pcg(self, b, tol=1e-6, max_iters=200, precond=True, force_iters=0):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros_like(b)
        it = C.c_int(0)
        ratio = C.c_double(0)
        st = lib().orc_pcg(self.h, _p(b), tol, max_iters, int(precond), force_iters, _p(x),
                           C.byref(it), C.byref(ratio))
        return x, dict(status=st, iters=it.value, ratio=ratio.value)


class Sim:
    """Oracle simulation of one body: positions and velocities are [N, 3]."""

    def __init__(self, w, opts: Opts | None = None):
        self.w = w
        self.opts = opts if opts is not None else default_opts()
        self._keep = [np.ascontiguousarray(w.rest, np.float64),
                      np.ascontiguousarray(w.inv_mass, np.float64),
                      np.ascontiguousarray(w.tets, np.int32),
                      np.ascontiguousarray(w.edges, np.int32),
                      np.ascontiguousarray(w.vol_tet, np.int32),
                      np.ascontiguousarray(w.arap_tet, np.int32),
                      np.ascontiguousarray(w.alpha, np.float64)]
        rest, im, tets, edges, vt, at, al = self._keep
        st = C.c_int(0)
        g = w.gravity
        self.s = lib().orc_sim_create(rest.shape[0], _p(rest), _p(im), tets.shape[0], _p(tets),
                                      edges.shape[0], _p(edges), vt.shape[0], _p(vt),
                                      at.shape[0], _p(at), _p(al),
                                      w.dt, g[0], g[1], g[2], C.byref(self.opts), C.byref(st))
        if not self.s:
            raise OracleError(st.value, "orc_sim_create")
        self.m = lib().orc_sim_rows(self.s)
        self.nnz = lib().orc_sim_nnz(self.s)

    def __del__(self):
        if getattr(self, "s", None):
            lib().orc_sim_free(self.s)
            self.s = None

    def pattern(self):
        rp = np.zeros(self.m + 1, np.int64)
        col = np.zeros(self.nnz, np.int32)
        lib().orc_sim_pattern(self.s, _p(rp), _p(col))
        return rp, col

    def constraints(self, pos):
        pos = np.ascontiguousarray(pos, np.float64)
        Cv = np.zeros(self.m)
        g = np.zeros((self.m, 4, 3))
        lib().orc_sim_constraints(self.s, _p(pos), _p(Cv), _p(g))
        return Cv, g

    def assemble(self, pos, lam=None):
        pos = np.ascontiguousarray(pos, np.float64)
        val = np.zeros(self.nnz)
        b = np.zeros(self.m)
        lam = None if lam is None else np.ascontiguousarray(lam, np.float64)
        lib().orc_sim_assemble(self.s, _p(pos), _p(lam), _p(val), _p(b))
        return val, b

    def step(self, pos, vel, n_iters, force_pcg=None):
        """One frame in place on pos/vel ([N,3] float64). Returns per-iteration stats."""
        assert pos.dtype == np.float64 and pos.flags.c_contiguous
        assert vel.dtype == np.float64 and vel.flags.c_contiguous
        bn = np.zeros(max(n_iters, 1))
        its = np.zeros(max(n_iters, 1), np.int32)
        ratio = np.zeros(max(n_iters, 1))
        setup = np.zeros(max(n_iters, 1), np.int32)
        fp = None if force_pcg is None else np.ascontiguousarray(force_pcg, np.int32)
        st = lib().orc_sim_step(self.s, _p(pos), _p(vel), n_iters, _p(bn), _p(its), _p(ratio),
                                _p(setup), _p(fp))
        return dict(status=st, bnorm=bn[:n_iters], pcg_iters=its[:n_iters],
                    ratio=ratio[:n_iters], setup=setup[:n_iters])

    def hier(self) -> Hier | None:
        h = lib().orc_sim_hier(self.s)
        return Hier(h, False) if h else None

    def lam(self):
        out = np.zeros(self.m)
        lib().orc_sim_get_lambda(self.s, _p(out))
        return out

    def matrix_values(self):
        out = np.zeros(self.nnz)
        lib().orc_sim_get_matrix_values(self.s, _p(out))
        return out

    def rhs(self):
        out = np.zeros(self.m)
        lib().orc_sim_get_rhs(self.s, _p(out))
        return out

    def set_frame(self, f: int):
        lib().orc_sim_set_frame(self.s, f)


def aggregate(rowptr, col, val, prio, theta=0.1, with_roots=False):
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    prio = np.ascontiguousarray(prio, np.uint64)
    agg = np.zeros(rowptr.shape[0] - 1, np.int32)
    roots = np.zeros(rowptr.shape[0] - 1, np.int32)
    na = lib().orc_aggregate(rowptr.shape[0] - 1, _p(rowptr), _p(col), _p(val), theta,
                             _p(prio), _p(agg), _p(roots))
    if with_roots:
        return agg, int(na), roots.astype(bool)
    return agg, int(na)


def color(rowptr, col, prio):
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    prio = np.ascontiguousarray(prio, np.uint64)
    c = np.zeros(rowptr.shape[0] - 1, np.int32)
    nc = lib().orc_color(rowptr.shape[0] - 1, _p(rowptr), _p(col), _p(prio), _p(c))
    return c, int(nc)


def positions(w):
    """[N,3] copies of the workload's initial positions and velocities."""
    return np.ascontiguousarray(w.x0.copy()), np.ascontiguousarray(w.v0.copy())


def closest_rotation(F):
    """The rotation nearest to the 3x3 matrix F (oracle's ARAP reading)."""
    F = np.ascontiguousarray(F, np.float64).reshape(3, 3)
    R = np.zeros((3, 3))
    lib().orc_closest_rotation(_p(F), _p(R))
    return R


def arap_eval(rest, x):
    """C = |F - R|_F^2 and its gradient [4, 3] for one tet (rest, x: [4, 3])."""
    rest = np.ascontiguousarray(rest, np.float64).reshape(4, 3)
    x = np.ascontiguousarray(x, np.float64).reshape(4, 3)
    c = C.c_double(0.0)
    g = np.zeros((4, 3))
    if not lib().orc_arap_eval(_p(rest), _p(x), C.byref(c), _p(g)):
        raise OracleError(1, "orc_arap_eval: singular rest shape")
    return c.value, g
