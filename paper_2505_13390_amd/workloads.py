"""Seeded synthetic workloads: tetrahedral beams and an ellipsoidal "muscle".

This module only builds inputs (meshes, masses, compliances, initial state).
It holds none of the solver's arithmetic, so both the FP64 CPU oracle and the
HIP library consume exactly the same arrays.

Random numbers come from a counter-based generator: SplitMix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
``mix64(seed, stream, i)`` salts the stream once and then mixes ``salt + i``,
so for a fixed (seed, stream) distinct indices give distinct outputs.

Streams: 0 jitter, 1 compliance, 6 batch sizes, 7 initial noise.
(2..5 are drawn by the solver itself: near-kernel start, aggregation priority,
colouring priority, power-method start.)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
BASE_SEED = 20250513


def splitmix64(z):
    """SplitMix64 output function applied to a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def mix64(seed: int, stream: int, idx):
    salt = splitmix64(np.uint64(((int(seed) << 8) | int(stream)) & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        return splitmix64(salt + np.asarray(idx, dtype=np.uint64))


def uniform01(seed: int, stream: int, idx):
    """Open-interval uniform in (0, 1): (top 53 bits + 0.5) * 2^-53."""
    h = mix64(seed, stream, idx)
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


@dataclass
class Workload:
    name: str
    rest: np.ndarray          # [N, 3] float64 rest positions
    inv_mass: np.ndarray      # [N] float64, 0 = pinned
    tets: np.ndarray          # [T, 4] int32, positively oriented
    edges: np.ndarray         # [E, 2] int32, i < j, lexicographic
    vol_tet: np.ndarray       # [V] int32 tet indices carrying a volume constraint
    alpha: np.ndarray         # [E + V + A] float64 compliance per constraint row
    dt: float
    gravity: tuple
    x0: np.ndarray            # [N, 3] float64 initial positions
    v0: np.ndarray            # [N, 3] float64 initial velocities
    frames: int = 1
    iters: int = 20
    info: dict = field(default_factory=dict)
    # [A] int32 tet indices carrying an ARAP constraint (rows after the volumes)
    arap_tet: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_rows(self) -> int:
        return int(self.edges.shape[0] + self.vol_tet.shape[0] + self.arap_tet.shape[0])


# --------------------------------------------------------------------------
# Lattice meshing (Kuhn / Freudenthal split: 6 tets per cube around the main
# diagonal, one per permutation of the axes; conforming across cubes).
# --------------------------------------------------------------------------
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _kuhn_tets(cells: np.ndarray, vid) -> np.ndarray:
    """cells: [C, 3] integer cube corners; vid(ijk [.,3]) -> vertex ids."""
    out = []
    for p in _PERMS:
        c0 = cells.copy()
        c1 = c0.copy(); c1[:, p[0]] += 1
        c2 = c1.copy(); c2[:, p[1]] += 1
        c3 = cells + 1
        t = np.stack([vid(c0), vid(c1), vid(c2), vid(c3)], axis=1)
        # orientation of the lattice tet: sign of det[e_p0, e_p0+e_p1, (1,1,1)]
        e1 = np.zeros(3); e1[p[0]] = 1
        e2 = e1.copy(); e2[p[1]] = 1
        sgn = np.linalg.det(np.stack([e1, e2, np.ones(3)]))
        if sgn < 0:
            t = t[:, [0, 1, 3, 2]]
        out.append(t)
    # interleave so that the 6 tets of one cube are contiguous
    return np.stack(out, axis=1).reshape(-1, 4).astype(np.int32)


def _unique_edges(tets: np.ndarray, n_verts: int) -> np.ndarray:
    pairs = []
    for a, b in [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]:
        i = tets[:, a].astype(np.int64)
        j = tets[:, b].astype(np.int64)
        pairs.append(np.minimum(i, j) * n_verts + np.maximum(i, j))
    key = np.unique(np.concatenate(pairs))
    return np.stack([key // n_verts, key % n_verts], axis=1).astype(np.int32)


def _jitter(seed: int, n: int, amp: float) -> np.ndarray:
    u = uniform01(seed, 0, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    return (2.0 * u - 1.0) * amp


def tet_volumes(pos: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Signed tet volumes via numpy determinants (input preparation only)."""
    a = pos[tets[:, 0]]
    m = np.stack([pos[tets[:, 1]] - a, pos[tets[:, 2]] - a, pos[tets[:, 3]] - a], axis=1)
    return np.linalg.det(m) / 6.0


def beam(nx: int, ny: int, nz: int, *, seed: int, volumes: bool, alpha_edge: float,
         alpha_vol: float = 0.0, dt: float = 1.0 / 60.0, jitter_frac: float = 1e-3,
         name: str = "beam") -> Workload:
    """Beam of nx*ny*nz unit cubes (long axis x), cell h = 1/ny, x=0 face pinned,
    unit mass per vertex, jittered lattice as the rest shape, at rest initially."""
    h = 1.0 / ny
    NX, NY, NZ = nx + 1, ny + 1, nz + 1
    ii, jj, kk = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    lat = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    n_verts = lat.shape[0]

    def vid(c):
        return (c[:, 0] * NY + c[:, 1]) * NZ + c[:, 2]

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    tets = _kuhn_tets(cells, vid)
    edges = _unique_edges(tets, n_verts)
    rest = lat.astype(np.float64) * h + _jitter(seed, n_verts, jitter_frac * h)
    inv_mass = np.where(lat[:, 0] == 0, 0.0, 1.0)
    vol_tet = np.arange(tets.shape[0], dtype=np.int32) if volumes else np.zeros(0, np.int32)
    alpha = np.concatenate([np.full(edges.shape[0], alpha_edge),
                            np.full(vol_tet.shape[0], alpha_vol)])
    return Workload(name=name, rest=rest, inv_mass=inv_mass, tets=tets, edges=edges,
                    vol_tet=vol_tet, alpha=alpha, dt=dt, gravity=(0.0, -9.8, 0.0),
                    x0=rest.copy(), v0=np.zeros_like(rest),
                    info={"grid": (nx, ny, nz), "h": h})


def arap_beam(nx: int, ny: int, nz: int, *, seed: int, mu: float = 1e9, dt: float = 0.01,
              squash: float = 0.3, jitter_frac: float = 1e-3, name: str = "arap_beam") -> Workload:
    """Soft-body beam with one ARAP row per tet (no edge or volume rows): the
    lattice and pinning of ``beam``, compliance 1 / (mu V_rest) per tet, and an
    initial state squashed by ``squash`` along the long axis towards the pinned
    x = 0 face, at rest velocity, which the constraints then restore."""
    b = beam(nx, ny, nz, seed=seed, volumes=False, alpha_edge=0.0, dt=dt,
             jitter_frac=jitter_frac, name=name)
    vol = tet_volumes(b.rest, b.tets)
    assert (vol > 0).all(), "jitter inverted a tet"
    x0 = b.rest.copy()
    x0[:, 0] *= 1.0 - squash
    return Workload(name=name, rest=b.rest, inv_mass=b.inv_mass, tets=b.tets,
                    edges=np.zeros((0, 2), np.int32), vol_tet=np.zeros(0, np.int32),
                    alpha=1.0 / (mu * vol), dt=dt, gravity=b.gravity, x0=x0,
                    v0=np.zeros_like(x0), arap_tet=np.arange(b.tets.shape[0], dtype=np.int32),
                    info={"grid": (nx, ny, nz), "h": b.info["h"], "mu": mu, "squash": squash})


def ellipsoid(nx: int, ny: int, nz: int, *, seed: int, semi=(0.5, 0.5, 1.0),
              density: float = 1000.0, jitter_cells: float = 0.2,
              name: str = "ellipsoid") -> Workload:
    """Ellipsoidal muscle: cubes of a cubic grid kept iff their centre lies inside
    the ellipsoid; seeded +-0.2 cell jitter defines the rest shape; masses lumped
    from rest tet volumes at the given density; edges + one volume row per tet."""
    h = 2.0 * semi[0] / nx
    assert abs(2.0 * semi[1] / ny - h) < 1e-12 and abs(2.0 * semi[2] / nz - h) < 1e-12
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    lo = -np.asarray(semi, dtype=np.float64)
    centre = lo + (cells + 0.5) * h
    inside = ((centre / np.asarray(semi)) ** 2).sum(axis=1) < 1.0
    cells = cells[inside]
    NX, NY, NZ = nx + 1, ny + 1, nz + 1

    def gid(c):
        return (c[:, 0].astype(np.int64) * NY + c[:, 1]) * NZ + c[:, 2]

    tets_g = _kuhn_tets(cells, gid).astype(np.int64)
    used = np.unique(tets_g)
    remap = -np.ones(NX * NY * NZ, dtype=np.int64)
    remap[used] = np.arange(used.shape[0])
    tets = remap[tets_g].astype(np.int32)
    n_verts = used.shape[0]
    gi = used // (NY * NZ)
    gj = (used // NZ) % NY
    gk = used % NZ
    lat = np.stack([gi, gj, gk], axis=1).astype(np.float64)
    rest = lo + lat * h + _jitter(seed, n_verts, jitter_cells * h)
    edges = _unique_edges(tets, n_verts)
    vol = tet_volumes(rest, tets)
    assert (vol > 0).all(), "jitter inverted a tet"
    mass = np.zeros(n_verts)
    np.add.at(mass, tets.ravel(), np.repeat(density * vol / 4.0, 4))
    inv_mass = 1.0 / mass
    vol_tet = np.arange(tets.shape[0], dtype=np.int32)
    m = edges.shape[0] + vol_tet.shape[0]
    u = uniform01(seed, 1, np.arange(m, dtype=np.uint64))
    alpha = np.exp(math.log(1e-10) + u * (math.log(1e-6) - math.log(1e-10)))
    return Workload(name=name, rest=rest, inv_mass=inv_mass, tets=tets, edges=edges,
                    vol_tet=vol_tet, alpha=alpha, dt=1.0 / 60.0, gravity=(0.0, -9.8, 0.0),
                    x0=rest.copy(), v0=np.zeros_like(rest),
                    info={"grid": (nx, ny, nz), "h": h})


# --------------------------------------------------------------------------
# The named workloads: the edge beam, the edge + volume beam, the muscle, the
# 64-beam batch, the stiff copies and the two ARAP beams.
# --------------------------------------------------------------------------
def beam_c0(seed: int = BASE_SEED + 0) -> Workload:
    """8x8x32 cube beam, edges only, compliance 1e-8, 1 frame x 20 iterations."""
    w = beam(32, 8, 8, seed=seed, volumes=False, alpha_edge=1e-8, name="beam_8x8x32_edges")
    w.frames, w.iters = 1, 20
    return w


def beam_c1(seed: int = BASE_SEED + 1) -> Workload:
    """32x32x128 cube beam, edges (1e-9) + volumes (1e-10), 10 frames x 20 iterations."""
    w = beam(128, 32, 32, seed=seed, volumes=True, alpha_edge=1e-9, alpha_vol=1e-10,
             name="beam_32x32x128_edges_volumes")
    w.frames, w.iters = 10, 20
    return w


def arap_a0(seed: int = BASE_SEED + 10) -> Workload:
    """8x8x32 ARAP beam (12,288 tet rows), mu 1e9, dt 10 ms, squashed 30%,
    1 frame x 20 iterations (the material of the paper's soft-body scenes)."""
    w = arap_beam(32, 8, 8, seed=seed, name="arap_beam_8x8x32")
    w.frames, w.iters = 1, 20
    return w


def arap_a1(seed: int = BASE_SEED + 11) -> Workload:
    """32x32x128 ARAP beam (786,432 tet rows), mu 1e9, dt 10 ms, squashed 30%,
    frames of 20 iterations."""
    w = arap_beam(128, 32, 32, seed=seed, name="arap_beam_32x32x128")
    w.frames, w.iters = 10, 20
    return w


def muscle_c2(seed: int = BASE_SEED + 2, grid=(64, 64, 128)) -> Workload:
    """Ellipsoidal muscle, cube-centre clip, pins |z| >= 0.9, gravity -y, 1 x 20."""
    w = ellipsoid(*grid, seed=seed, name="ellipsoid_%dx%dx%d" % grid)
    w.inv_mass = np.where(np.abs(w.rest[:, 2]) >= 0.9, 0.0, w.inv_mass)
    w.frames, w.iters = 1, 20
    return w


def batch_c3(seed: int = BASE_SEED + 3, count: int = 64, lo: int = 4, hi: int = 24):
    """64 beams n x n x 4n, n = round(exp(U(ln lo, ln hi))), edges + volumes at 1e-8."""
    u = uniform01(seed, 6, np.arange(count, dtype=np.uint64))
    ns = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(int)
    out = []
    for k, n in enumerate(ns):
        w = beam(4 * int(n), int(n), int(n), seed=seed * 1000 + k, volumes=True,
                 alpha_edge=1e-8, alpha_vol=1e-8, name="beam_%d" % n)
        w.frames, w.iters = 10, 20
        out.append(w)
    return out


def stiff_c4(seed: int = BASE_SEED + 4, grid=(64, 64, 128), copies: int = 8):
    """Stiff large-step test: the muscle mesh, compliance 1e-12, dt 1/30, free body
    without gravity, compressed to 70% along its long axis plus 1e-3 h noise."""
    base = ellipsoid(*grid, seed=BASE_SEED + 2, name="ellipsoid_stiff")
    out = []
    for c in range(copies):
        w = Workload(**{k: getattr(base, k) for k in base.__dataclass_fields__})
        w.rest = base.rest.copy()
        w.alpha = np.full(base.alpha.shape[0], 1e-12)
        w.dt = 1.0 / 30.0
        w.gravity = (0.0, 0.0, 0.0)
        h = base.info["h"]
        x0 = base.rest.copy()
        zc = x0[:, 2].mean()
        x0[:, 2] = zc + 0.7 * (x0[:, 2] - zc)
        n = x0.shape[0]
        u = uniform01(seed * 100 + c, 7, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
        x0 += (2.0 * u - 1.0) * 1e-3 * h
        w.x0 = x0
        w.v0 = np.zeros_like(x0)
        w.frames, w.iters = 50, 20
        out.append(w)
    return out


def tiny_beam(nx: int = 2, ny: int = 1, nz: int = 1, *, volumes: bool = True, seed: int = 7,
              alpha_edge: float = 1e-6, alpha_vol: float = 1e-6, pin: bool = True,
              jitter_frac: float = 1e-3) -> Workload:
    """Small beams for closed-form and dense checks."""
    w = beam(nx, ny, nz, seed=seed, volumes=volumes, alpha_edge=alpha_edge,
             alpha_vol=alpha_vol, jitter_frac=jitter_frac, name="tiny_%dx%dx%d" % (nx, ny, nz))
    if not pin:
        w.inv_mass = np.ones_like(w.inv_mass)
    return w


def perturbed(w: Workload, amp: float, seed: int = 99) -> Workload:
    """Copy of w with initial positions displaced by a seeded uniform +-amp."""
    n = w.n_verts
    u = uniform01(seed, 7, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    x0 = w.rest + (2.0 * u - 1.0) * amp
    x0[w.inv_mass == 0] = w.rest[w.inv_mass == 0]
    v = Workload(**{k: getattr(w, k) for k in w.__dataclass_fields__})
    v.x0 = x0
    v.v0 = np.zeros_like(x0)
    return v


CONFIGS = {"C0": beam_c0, "C1": beam_c1, "C2": muscle_c2, "A0": arap_a0, "A1": arap_a1}
