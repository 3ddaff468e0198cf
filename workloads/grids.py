"""Grids, metrics, models and traveltimes for the synthetic workloads.

Index conventions (shared by every consumer):
  * node id n = i + n1*(j + n2*k) with i (logical xi) fastest; a 2-D grid uses
    axes (i, k) with n2 = 1, so n = i + n1*k;
  * arrays over the grid are shaped (n3, n2, n1) in 3-D and (n3, n1) in 2-D
    before flattening;
  * G is [N][6] = (Gxx, Gyy, Gzz, Gxy, Gxz, Gyz) in 3-D and [N][3] =
    (Gxx, Gzz, Gxz) in 2-D, in logical index units (unit spacing per index);
  * batched vectors are [N][B] (right-hand side fastest).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfmgen.so")
_lib = None

CONFIG_NAMES = ("c1", "c2", "c3", "c4")


def build(verbose: bool = False) -> str:
    """Compile the first-arrival generator (plain C, OpenMP) in place."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH,
           os.path.join(_HERE, "eikonal.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.fmgen_eikonal.restype = ctypes.c_int
        lib.fmgen_eikonal.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
        lib.fmgen_eikonal_pt.restype = ctypes.c_int
        lib.fmgen_eikonal_pt.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Workload:
    """A frozen-transport problem: grid, metric, slowness, sources, receivers."""
    name: str
    dim: int
    n1: int
    n2: int
    n3: int
    X: np.ndarray          # [N][dim] physical node coordinates
    G: np.ndarray          # [N][3] or [N][6] metric in index units
    s: np.ndarray          # [N] slowness
    src: np.ndarray        # [S] int64 source node ids
    rcv: np.ndarray        # [R] int64 receiver node ids (shared by all sources)
    B: int = 1             # right-hand sides per source
    seed: int = 0
    T: np.ndarray | None = None   # [S][N] background traveltime
    meta: dict = field(default_factory=dict)
    # interpolating receivers: rcv is then [R][K] nodes and rcv_w [R][K]
    # weights (receiver r samples sum_k rcv_w[r][k] x[rcv[r][k]])
    rcv_w: np.ndarray | None = None

    @property
    def N(self) -> int:
        return self.n1 * self.n2 * self.n3

    @property
    def S(self) -> int:
        return int(self.src.shape[0])

    @property
    def shape(self):
        return (self.n3, self.n2, self.n1) if self.dim == 3 else (self.n3, self.n1)

    def node(self, i, j, k):
        return i + self.n1 * (j + self.n2 * k)


# --------------------------------------------------------------------------
# metric
# --------------------------------------------------------------------------

def metric_from_coords(X: np.ndarray, dim: int) -> np.ndarray:
    """G = J^{-1} J^{-T} from node coordinates (Section 2.2, eq. (metric-eikonal)).

    X is shaped grid_shape + (dim,).  J_ab = dx_a / dxi_b is taken by
    second-order differences in index space (one-sided second order on the
    boundary), so G is in logical index units.
    """
    grid_shape = X.shape[:-1]
    N = int(np.prod(grid_shape))
    # axis order in the array is (k, j, i) or (k, i); logical axis b maps to
    # array axis dim-1-b
    J = np.empty(grid_shape + (dim, dim))
    for b in range(dim):
        ax = dim - 1 - b
        for a in range(dim):
            J[..., a, b] = np.gradient(X[..., a], axis=ax, edge_order=2)
    J = J.reshape(N, dim, dim)
    Ji = np.linalg.inv(J)
    Gm = Ji @ np.transpose(Ji, (0, 2, 1))
    if dim == 3:
        return np.ascontiguousarray(np.stack(
            [Gm[:, 0, 0], Gm[:, 1, 1], Gm[:, 2, 2], Gm[:, 0, 1], Gm[:, 0, 2], Gm[:, 1, 2]], axis=1))
    return np.ascontiguousarray(np.stack([Gm[:, 0, 0], Gm[:, 1, 1], Gm[:, 0, 1]], axis=1))


def jacobian_det(X: np.ndarray, dim: int) -> np.ndarray:
    grid_shape = X.shape[:-1]
    J = np.empty(grid_shape + (dim, dim))
    for b in range(dim):
        ax = dim - 1 - b
        for a in range(dim):
            J[..., a, b] = np.gradient(X[..., a], axis=ax, edge_order=2)
    return np.linalg.det(J.reshape(-1, dim, dim))


def mu_g(G: np.ndarray, dim: int) -> float:
    """Cross-metric strength, eq. (muG)."""
    if dim == 3:
        gxx, gyy, gzz, gxy, gxz, gyz = (G[:, c] for c in range(6))
        r = np.maximum.reduce([np.abs(gxy) / np.sqrt(gxx * gyy),
                               np.abs(gxz) / np.sqrt(gxx * gzz),
                               np.abs(gyz) / np.sqrt(gyy * gzz)])
    else:
        gxx, gzz, gxz = (G[:, c] for c in range(3))
        r = np.abs(gxz) / np.sqrt(gxx * gzz)
    return float(r.max())


# --------------------------------------------------------------------------
# first-arrival traveltimes
# --------------------------------------------------------------------------

def eikonal(wl: Workload, init_radius: int = 2, nthreads: int | None = None) -> np.ndarray:
    """First-arrival traveltimes [S][N] for every source of the workload."""
    lib = _load()
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    N = wl.N
    T = np.empty((wl.S, N), dtype=np.float64)
    G = np.ascontiguousarray(wl.G, dtype=np.float64)
    X = np.ascontiguousarray(wl.X, dtype=np.float64)
    s = np.ascontiguousarray(wl.s, dtype=np.float64)
    src = np.ascontiguousarray(wl.src, dtype=np.int64)
    rc = lib.fmgen_eikonal(wl.dim, wl.n1, wl.n2, wl.n3, G.ctypes.data, X.ctypes.data,
                           s.ctypes.data, wl.S, src.ctypes.data, init_radius, nthreads,
                           T.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"fmgen_eikonal failed with code {rc}")
    wl.T = T
    return T


def eikonal_point(wl: Workload, xi: np.ndarray, rho: float, nthreads: int | None = None) -> np.ndarray:
    """First-arrival traveltimes [S][N] for off-grid point sources at logical
    coordinates xi [S][dim], seed region of max-norm radius rho (straight-ray
    times there, fast marching elsewhere); sets wl.T."""
    lib = _load()
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, wl.dim)
    S = xi.shape[0]
    T = np.empty((S, wl.N), dtype=np.float64)
    G = np.ascontiguousarray(wl.G, dtype=np.float64)
    X = np.ascontiguousarray(wl.X, dtype=np.float64)
    s = np.ascontiguousarray(wl.s, dtype=np.float64)
    rc = lib.fmgen_eikonal_pt(wl.dim, wl.n1, wl.n2, wl.n3, G.ctypes.data, X.ctypes.data, s.ctypes.data, S,
                              xi.ctypes.data, float(rho), nthreads, T.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"fmgen_eikonal_pt failed with code {rc}")
    wl.T = T
    return T


def traveltime_solver(wl: Workload, init_radius: int = 2, nthreads: int | None = None):
    """A callable s -> T[S][N]: the first-arrival generator for this grid,
    sources and a given slowness field."""
    import copy

    def solve(s):
        w2 = copy.copy(wl)
        w2.s = np.ascontiguousarray(s, dtype=np.float64)
        return eikonal(w2, init_radius=init_radius, nthreads=nthreads)
    return solve


def perturbed_model(wl: Workload, seed: int, n: int = 6, amp: float = 0.05, sigma_km: float = 0.4) -> np.ndarray:
    """A "true" slowness for a Gauss-Newton test: s * (1 + sum of n seeded
    Gaussian anomalies of relative amplitude U[-amp, amp] and width sigma_km,
    centred inside the domain)."""
    rng = np.random.default_rng(seed)
    X = wl.X
    lo, hi = X.min(axis=0), X.max(axis=0)
    f = np.zeros(X.shape[0])
    for _ in range(n):
        c = lo + (0.2 + 0.6 * rng.random(X.shape[1])) * (hi - lo)
        a = rng.uniform(-amp, amp)
        f += a * np.exp(-np.sum((X - c) ** 2, axis=1) / (2 * sigma_km ** 2))   # coordinates in km
    return wl.s * (1.0 + f)


# --------------------------------------------------------------------------
# seeded vectors
# --------------------------------------------------------------------------

def _box5(a: np.ndarray, axes) -> np.ndarray:
    out = a
    for ax in axes:
        pad = [(0, 0)] * out.ndim
        pad[ax] = (2, 2)
        p = np.pad(out, pad, mode="edge")
        n = out.shape[ax]
        acc = np.zeros_like(out)
        for o in range(5):
            acc += np.take(p, np.arange(o, o + n), axis=ax)
        out = acc / 5.0
    return out


def smooth_noise(wl: Workload, B: int, rng: np.random.Generator, rel_rms: float = 0.01) -> np.ndarray:
    """Slowness perturbations [N][B]: Gaussian noise smoothed by a separable
    5-node box filter (edge replication), scaled to rel_rms * RMS(s) per column."""
    shape = wl.shape
    a = rng.standard_normal(shape + (B,))
    a = _box5(a, range(len(shape)))
    a = a.reshape(wl.N, B)
    rms_s = np.sqrt(np.mean(wl.s ** 2))
    a *= rel_rms * rms_s / np.sqrt(np.mean(a ** 2, axis=0, keepdims=True))
    return np.ascontiguousarray(a)


def data_noise(shape, rng: np.random.Generator) -> np.ndarray:
    return np.ascontiguousarray(rng.standard_normal(shape))


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def cell_velocities(wl: Workload) -> np.ndarray:
    """A cell-velocity model from the workload's nodal slowness: each cell
    (hexahedron, or quadrilateral in 2-D, between logical neighbours; cell id
    ci + (n1-1) (cj + (n2-1) ck)) gets the mean of 1/s over its corners."""
    v = 1.0 / np.asarray(wl.s, dtype=np.float64)
    if wl.dim == 3:
        g = v.reshape(wl.n3, wl.n2, wl.n1)
        c = sum(g[k:k + wl.n3 - 1, j:j + wl.n2 - 1, i:i + wl.n1 - 1]
                for k in (0, 1) for j in (0, 1) for i in (0, 1)) / 8.0
    else:
        g = v.reshape(wl.n3, wl.n1)
        c = sum(g[k:k + wl.n3 - 1, i:i + wl.n1 - 1] for k in (0, 1) for i in (0, 1)) / 4.0
    return np.ascontiguousarray(c.reshape(-1))


def interpolating_receivers(wl: Workload, R: int, seed: int):
    """R receivers at seeded points of the surface (logical k = 0) between
    nodes: logical coordinates uniform over the surface, each receiver
    sampling the bilinear (3-D, 4 nodes) or linear (2-D, 2 nodes) interpolant
    of the surface cell around it, in logical coordinates.  Returns
    (nodes [R][K] int64, weights [R][K], coordinates [R][dim-1])."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(0.0, wl.n1 - 1, R)
    i0 = np.minimum(np.floor(xi).astype(np.int64), wl.n1 - 2)
    fx = xi - i0
    if wl.dim == 2:
        nodes = np.stack([i0, i0 + 1], axis=1)
        w = np.stack([1.0 - fx, fx], axis=1)
        return nodes, w, xi[:, None]
    eta = rng.uniform(0.0, wl.n2 - 1, R)
    j0 = np.minimum(np.floor(eta).astype(np.int64), wl.n2 - 2)
    fy = eta - j0
    n1 = wl.n1
    nodes = np.stack([i0 + n1 * j0, i0 + 1 + n1 * j0, i0 + n1 * (j0 + 1), i0 + 1 + n1 * (j0 + 1)], axis=1)
    w = np.stack([(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy), (1.0 - fx) * fy, fx * fy], axis=1)
    return nodes, w, np.stack([xi, eta], axis=1)


def _lattice(n: int, m: int) -> np.ndarray:
    return np.rint((np.arange(m) + 0.5) * (n - 1) / m).astype(np.int64)


def _mk(name, dim, n1, n2, n3, X, s, src, rcv, B, seed, meta=None) -> Workload:
    G = metric_from_coords(X, dim)
    N = n1 * n2 * n3
    return Workload(name=name, dim=dim, n1=n1, n2=n2, n3=n3,
                    X=np.ascontiguousarray(X.reshape(N, dim)), G=G,
                    s=np.ascontiguousarray(s.reshape(N)),
                    src=np.asarray(src, dtype=np.int64), rcv=np.asarray(rcv, dtype=np.int64),
                    B=B, seed=seed, meta=meta or {})


def deformed_2d(n1: int, n3: int, seed: int, topo_amp: float, n_anom: int,
                S: int, B: int, R: int, name: str) -> Workload:
    """2-D family: x = 4 km * xi, z = h(xi) + zeta (2 km - h(xi)), depth z
    positive downward; v = 1.5 + 0.8 z km/s with seeded +-15 % Gaussian
    anomalies of radius 0.3 km; h = topo_amp sin(2 pi xi / 1.5) plus four seeded
    Gaussian bumps of amplitude U[-50, 50] m and width 0.2 km."""
    rng = np.random.default_rng(seed)
    xi = np.linspace(0.0, 1.0, n1)
    ze = np.linspace(0.0, 1.0, n3)
    x1 = 4.0 * xi
    h = topo_amp * np.sin(2.0 * np.pi * xi / 1.5)
    for _ in range(4):
        a = rng.uniform(-0.05, 0.05)
        c = 4.0 * rng.uniform(0.1, 0.9)
        h = h + a * np.exp(-(x1 - c) ** 2 / (2.0 * 0.2 ** 2))
    Z = h[None, :] + ze[:, None] * (2.0 - h[None, :])
    Xc = np.broadcast_to(x1[None, :], Z.shape)
    X = np.stack([Xc, Z], axis=-1)
    v = 1.5 + 0.8 * Z
    for _ in range(n_anom):
        amp = 0.15 * (1.0 if rng.uniform() < 0.5 else -1.0)
        cx = rng.uniform(1.0, 3.0) if n_anom == 1 else rng.uniform(0.5, 3.5)
        cz = rng.uniform(0.5, 1.5) if n_anom == 1 else rng.uniform(0.4, 1.6)
        r2 = (Xc - cx) ** 2 + (Z - cz) ** 2
        v = v * (1.0 + amp * np.exp(-r2 / (2.0 * 0.3 ** 2)))
    s = 1.0 / v
    if S == 1:
        src_i = np.array([int(rng.integers(n1 // 8, 7 * n1 // 8))])
    else:
        src_i = _lattice(n1, S)
    src = src_i  # k = 0 surface
    rcv = _lattice(n1, R)
    return _mk(name, 2, n1, 1, n3, X, s, src, rcv, B, seed,
               meta={"topo_amp_km": topo_amp, "anomalies": n_anom})


def deformed_3d(n1: int, n2: int, n3: int, seed: int, Sx: int, Sy: int, B: int,
                Rx: int, Ry: int, name: str) -> Workload:
    """3-D family on a 4 x 4 x 2 km domain: z = h(x,y) + zeta (2 km - h), h a sum
    of three seeded 2-D sinusoids scaled to max |h| = 0.3 km; v = (1.8 + 0.6 z)
    (1 + 0.1 sin(pi (x-px)/0.5) sin(pi (y-py)/0.5) sin(pi (z-pz)/0.5)) km/s, a
    smooth checkerboard of 0.5 km cells with a seeded phase."""
    rng = np.random.default_rng(seed)
    xi = np.linspace(0.0, 1.0, n1)
    et = np.linspace(0.0, 1.0, n2)
    ze = np.linspace(0.0, 1.0, n3)
    x1 = 4.0 * xi
    y1 = 4.0 * et
    XX, YY = np.meshgrid(x1, y1, indexing="xy")   # shape (n2, n1)
    h = np.zeros_like(XX)
    for _ in range(3):
        kx = rng.integers(1, 4) * (1 if rng.uniform() < 0.5 else -1)
        ky = rng.integers(1, 4)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        amp = rng.uniform(0.5, 1.0)
        h = h + amp * np.sin(2.0 * np.pi * (kx * XX + ky * YY) / 4.0 + ph)
    h *= 0.3 / np.abs(h).max()
    Z = h[None, :, :] + ze[:, None, None] * (2.0 - h[None, :, :])
    Xc = np.broadcast_to(XX[None], Z.shape)
    Yc = np.broadcast_to(YY[None], Z.shape)
    X = np.stack([Xc, Yc, Z], axis=-1)
    px, py, pz = rng.uniform(0.0, 1.0, 3)
    chk = (np.sin(np.pi * (Xc - px) / 0.5) * np.sin(np.pi * (Yc - py) / 0.5)
           * np.sin(np.pi * (Z - pz) / 0.5))
    v = (1.8 + 0.6 * Z) * (1.0 + 0.1 * chk)
    s = 1.0 / v
    si, sj = _lattice(n1, Sx), _lattice(n2, Sy)
    src = np.array([i + n1 * j for j in sj for i in si], dtype=np.int64)
    ri, rj = _lattice(n1, Rx), _lattice(n2, Ry)
    rcv = np.array([i + n1 * j for j in rj for i in ri], dtype=np.int64)
    return _mk(name, 3, n1, n2, n3, X, s, src, rcv, B, seed)


def config(name: str, with_T: bool = True, nthreads: int | None = None) -> Workload:
    """The benchmark configurations c1..c4 (c5 shares c4's grid)."""
    if name == "c1":
        wl = deformed_2d(81, 41, 1000, 0.2, 1, S=1, B=1, R=81, name="c1")
    elif name == "c2":
        wl = deformed_2d(401, 201, 2000, 0.4, 5, S=16, B=32, R=100, name="c2")
    elif name == "c3":
        wl = deformed_3d(101, 101, 51, 3000, Sx=4, Sy=2, B=16, Rx=10, Ry=10, name="c3")
    elif name == "c4":
        wl = deformed_3d(201, 201, 101, 4000, Sx=8, Sy=8, B=16, Rx=20, Ry=20, name="c4")
    else:
        raise ValueError(name)
    if with_T:
        eikonal(wl, nthreads=nthreads)
    return wl


def smooth_3d(n1: int, n2: int, n3: int, topo_amp: float = 0.0, name: str = "smooth3d",
              with_T: bool = True) -> Workload:
    """A smooth 3-D member for refinement studies, the same physical problem
    at every size: 4 x 4 x 2 km, surface h = topo_amp sin(2 pi x / 4) cos(2 pi y / 4)
    km, v = 1.8 + 0.6 z km/s, one source at the centre of the surface lattice
    and 5 x 5 surface receivers (the lattices scale with the grid)."""
    xi = np.linspace(0.0, 1.0, n1)
    et = np.linspace(0.0, 1.0, n2)
    ze = np.linspace(0.0, 1.0, n3)
    XX, YY = np.meshgrid(4.0 * xi, 4.0 * et, indexing="xy")
    h = topo_amp * np.sin(2.0 * np.pi * XX / 4.0) * np.cos(2.0 * np.pi * YY / 4.0)
    Z = h[None, :, :] + ze[:, None, None] * (2.0 - h[None, :, :])
    X = np.stack([np.broadcast_to(XX[None], Z.shape), np.broadcast_to(YY[None], Z.shape), Z], axis=-1)
    s = 1.0 / (1.8 + 0.6 * Z)
    si, sj = _lattice(n1, 1), _lattice(n2, 1)
    src = np.array([i + n1 * j for j in sj for i in si], dtype=np.int64)
    ri, rj = _lattice(n1, 5), _lattice(n2, 5)
    rcv = np.array([i + n1 * j for j in rj for i in ri], dtype=np.int64)
    wl = _mk(name, 3, n1, n2, n3, X, s, src, rcv, 1, 0, meta={"topo_amp": topo_amp})
    if with_T:
        eikonal(wl)
    return wl


def small_3d(n1: int, n2: int, n3: int, seed: int, S: int, B: int, name: str = "small3d",
             with_T: bool = True) -> Workload:
    """A reduced member of the 3-D family (same recipe, fewer nodes)."""
    sx = int(np.ceil(np.sqrt(S)))
    sy = int(np.ceil(S / sx))
    wl = deformed_3d(n1, n2, n3, seed, Sx=sx, Sy=sy, B=B, Rx=5, Ry=5, name=name)
    wl.src = wl.src[:S]
    if with_T:
        eikonal(wl)
    return wl


# --------------------------------------------------------------------------
# analytic fixtures of Section 5
# --------------------------------------------------------------------------

def _test_map(n1, n2, n3, L, H, A):
    """eq. (test-map)/(test-topo): x = xi, y = eta, z = zeta + (1 - zeta/H) h."""
    xi = np.linspace(-L / 2, L / 2, n1)
    et = np.linspace(-L / 2, L / 2, n2)
    ze = np.linspace(0.0, H, n3)
    K, Jg, I = np.meshgrid(ze, et, xi, indexing="ij")
    h = A * np.sin(2.0 * np.pi * I / L) * np.sin(2.0 * np.pi * Jg / L)
    Z = K + (1.0 - K / H) * h
    return np.stack([I, Jg, Z], axis=-1)


def manufactured(n1: int, n2: int, n3: int, A: float = 200.0, v0: float = 3000.0):
    """Point-source tangent test of Section 5.1: analytic T = s0 r at the nodes of
    the sinusoidal-surface grid, source at the centre logical node.  Returns
    the workload plus (dS, dT_exact) for eq. (test-ds) and eq. (test-dT)."""
    L, H = 4000.0, 2000.0
    X = _test_map(n1, n2, n3, L, H, A)
    s0 = 1.0 / v0
    s = np.full(X.shape[:-1], s0)
    src = (n1 // 2) + n1 * ((n2 // 2) + n2 * (n3 // 2))
    wl = _mk(f"manufactured{n1}x{n2}x{n3}", 3, n1, n2, n3, X, s, [src], [], 1, 0,
             meta={"A": A, "v0": v0, "L": L, "H": H})
    xs = wl.X[src]
    r = np.linalg.norm(wl.X - xs[None, :], axis=1)
    wl.T = (s0 * r)[None, :]
    c0, cx, cy, cz = 0.02, 0.04, -0.03, 0.02
    ds = s0 * (c0 + cx * (wl.X[:, 0] - xs[0]) / L + cy * (wl.X[:, 1] - xs[1]) / L
               + cz * (wl.X[:, 2] - xs[2]) / H)
    ds_src = s0 * c0
    dT = 0.5 * r * (ds_src + ds)
    wl.meta.update({"h": max(L / (n1 - 1), L / (n2 - 1), H / (n3 - 1)), "r": r})
    return wl, ds, dT


def flat_radial(n1: int, n2: int, n3: int, v0: float = 3000.0, src_ijk=None):
    """Flat grid (A = 0) with radial traveltime, eq. (radial-state)."""
    L, H = 4000.0, 2000.0
    X = _test_map(n1, n2, n3, L, H, 0.0)
    s = np.full(X.shape[:-1], 1.0 / v0)
    if src_ijk is None:
        src_ijk = (n1 // 2, n2 // 2, 0)
    i, j, k = src_ijk
    src = i + n1 * (j + n2 * k)
    wl = _mk(f"flat{n1}x{n2}x{n3}", 3, n1, n2, n3, X, s, [src], [], 1, 0)
    r = np.linalg.norm(wl.X - wl.X[src][None, :], axis=1)
    wl.T = (r / v0)[None, :]
    return wl


def curved_state(n1: int = 41, n2: int = 41, n3: int = 25, A: float = 500.0,
                 eps_T: float = 0.05, v0: float = 3000.0, src_ijk=None, radial: bool = False):
    """Controlled dependency-regime fixture of Section 5.2: surface of
    eq. (graph-map), traveltime of eq. (curved-state) (or eq. (radial-state)
    when radial), slowness s = |grad_x T| from the analytic gradient."""
    L, H = 4000.0, 2000.0
    X = _test_map(n1, n2, n3, L, H, A)
    if src_ijk is None:
        src_ijk = ((n1 - 1) // 4, (n2 - 1) // 4, 0)   # quarter source on the surface
    i, j, k = src_ijk
    src = i + n1 * (j + n2 * k)
    Xf = X.reshape(-1, 3)
    xs = Xf[src]
    d = Xf - xs[None, :]
    r = np.linalg.norm(d, axis=1)
    x, y, z = Xf[:, 0], Xf[:, 1], Xf[:, 2]
    Xs, Ys = x + L / 2, y + L / 2
    if radial or eps_T == 0.0:
        T = r / v0
        gx = d[:, 0] / np.where(r > 0, r, 1.0) / v0
        gy = d[:, 1] / np.where(r > 0, r, 1.0) / v0
        gz = d[:, 2] / np.where(r > 0, r, 1.0) / v0
    else:
        k4 = 4.0 * np.pi / L
        sx, cx_ = np.sin(k4 * Xs), np.cos(k4 * Xs)
        sy, cy_ = np.sin(k4 * Ys), np.cos(k4 * Ys)
        sz, cz_ = np.sin(np.pi * z / H), np.cos(np.pi * z / H)
        pert = eps_T * sx * sy * sz
        T = r / v0 + pert
        T = T - T[src]
        rr = np.where(r > 0, r, 1.0)
        gx = d[:, 0] / rr / v0 + eps_T * k4 * cx_ * sy * sz
        gy = d[:, 1] / rr / v0 + eps_T * k4 * sx * cy_ * sz
        gz = d[:, 2] / rr / v0 + eps_T * (np.pi / H) * sx * sy * cz_
    s = np.sqrt(gx * gx + gy * gy + gz * gz)
    s[src] = 1.0 / v0
    wl = _mk(f"curved{n1}x{n2}x{n3}_A{A:g}_e{eps_T:g}", 3, n1, n2, n3, X, s, [src], [], 1, 0,
             meta={"A": A, "eps_T": eps_T})
    wl.T = T[None, :].copy()
    wl.T[0, src] = 0.0
    return wl
