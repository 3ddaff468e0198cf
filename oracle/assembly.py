"""Explicit assembly of the frozen transport operator (oracle; test infrastructure).

Follows Section 3.1 (face-based upwinding, eq. (discrete-row) and
eq. (transport-system)) and Section 3.2 (scale-consistent right-hand side).
Readings where the paper defers to an uncited reference or is silent:

  * face averages (the paper points to an external discretisation): for the face
    between p and p+e_d, G_f = (G_p + G_{p+e_d})/2, the normal derivative is the
    compact difference g_d = T_{p+e_d} - T_p, and each tangential derivative is
    the mean of the nodal central differences at p and p+e_d (one-sided on the
    first and last node of an axis); a_f = sum_{d'} (G_f)_{d d'} g_{d'} summed in
    axis order;
  * coupling: the minus face of p contributes c = max(a_f, 0) from p-e_d, the
    plus face contributes c = max(-a_f, 0) from p+e_d; an edge exists iff the
    normalised weight is strictly positive (Section 3.3);
  * the source row and rows without inflow are identity rows; the calibration
    c_i = l_i / s_i with l = A T then gives c_src = 0 (T_src = 0) and
    c_i = T_i / s_i on inflow-less rows.

The 26-neighbour (cube) stencil (cube_couplings) is a variant the paper does
not define: the same row form and calibration with upstream couplings that
interpolate along the node's backward characteristic on its 3x3x3 cube.

All sums are evaluated left to right in a fixed order (axis order for a_f,
slot order minus/plus per axis for d_p and for (W T)_p), with no fused
multiply-add, so the sign of every a_f is a deterministic FP64 decision.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def _grid_shape(dim, n1, n2, n3):
    return (n3, n2, n1) if dim == 3 else (n3, n1)


def _metric_full(G, dim, shape):
    """Per-node symmetric metric as a dim x dim nested list of grid arrays."""
    if dim == 3:
        gxx, gyy, gzz, gxy, gxz, gyz = (G[:, c].reshape(shape) for c in range(6))
        return [[gxx, gxy, gxz], [gxy, gyy, gyz], [gxz, gyz, gzz]]
    gxx, gzz, gxz = (G[:, c].reshape(shape) for c in range(3))
    return [[gxx, gxz], [gxz, gzz]]


def _sl(ndim, ax, s):
    idx = [slice(None)] * ndim
    idx[ax] = s
    return tuple(idx)


def _central(T, ax):
    """Nodal derivative along array axis ax: central in the interior, one-sided
    at the first and last node; zero if the axis has a single node."""
    n = T.shape[ax]
    D = np.zeros_like(T)
    if n == 1:
        return D
    nd = T.ndim
    D[_sl(nd, ax, 0)] = T[_sl(nd, ax, 1)] - T[_sl(nd, ax, 0)]
    D[_sl(nd, ax, n - 1)] = T[_sl(nd, ax, n - 1)] - T[_sl(nd, ax, n - 2)]
    if n > 2:
        D[_sl(nd, ax, slice(1, n - 1))] = 0.5 * (T[_sl(nd, ax, slice(2, n))]
                                                 - T[_sl(nd, ax, slice(0, n - 2))])
    return D


def face_coefficients(dim, n1, n2, n3, G, T):
    """a_f for every interior face, per logical axis d.

    Returns a list over d of arrays shaped like the grid with n_d - 1 entries
    along that axis: entry at p is the face between p and p + e_d.  Also
    returns the face derivative vectors g (list over d of lists over d').
    Section 3.1: the signed coefficient -a_f selects the upstream side.
    """
    shape = _grid_shape(dim, n1, n2, n3)
    Tg = np.asarray(T, dtype=np.float64).reshape(shape)
    Gm = _metric_full(np.asarray(G, dtype=np.float64), dim, shape)
    nd = len(shape)
    D = [_central(Tg, nd - 1 - dd) for dd in range(dim)]
    a_faces, g_faces = [], []
    for d in range(dim):
        ax = nd - 1 - d
        n = shape[ax]
        lo = _sl(nd, ax, slice(0, n - 1))
        hi = _sl(nd, ax, slice(1, n))
        g = []
        for dp in range(dim):
            if dp == d:
                g.append(Tg[hi] - Tg[lo])
            else:
                g.append(0.5 * (D[dp][lo] + D[dp][hi]))
        a = None
        for dp in range(dim):
            Gf = 0.5 * (Gm[d][dp][lo] + Gm[d][dp][hi])
            term = Gf * g[dp]
            a = term if a is None else a + term
        a_faces.append(a)
        g_faces.append(g)
    return a_faces, g_faces


@dataclass
class OracleOperator:
    """A = I - W (CSR, natural node order, row i holds w_ij for edges j -> i),
    calibration c, receivers, and the grid description."""
    dim: int
    n1: int
    n2: int
    n3: int
    W: sp.csr_matrix
    c: np.ndarray
    src: int
    rcv: np.ndarray
    T: np.ndarray
    s: np.ndarray
    rcv_w: np.ndarray | None = None

    @property
    def N(self):
        return self.n1 * self.n2 * self.n3

    def P(self) -> sp.csr_matrix:
        """The receiver sampling P_alpha (Section 4.4) as an R x N matrix:
        row r holds weight w[r][k] at node rcv[r][k] (entries at one node
        added); on-grid receivers, rcv of shape [R] without weights, give the
        selection rows e_rcv[r]."""
        nodes = np.asarray(self.rcv, dtype=np.int64)
        if nodes.ndim == 1:
            nodes = nodes[:, None]
        w = np.ones(nodes.shape) if self.rcv_w is None else np.asarray(self.rcv_w, dtype=np.float64)
        R, K = nodes.shape
        rows = np.repeat(np.arange(R), K)
        return sp.csr_matrix((w.reshape(-1), (rows, nodes.reshape(-1))), shape=(R, self.N))

    def A(self):
        return (sp.identity(self.N, format="csr") - self.W).tocsr()

    def WT(self):
        return self.W.T.tocsr()


def node_directions(dim, n1, n2, n3, G, T):
    """a = G grad_xi T at every node from the nodal metric and the nodal
    derivatives (central inside, one-sided on the first and last node of an
    axis), summed over d' in axis order; [N, dim], logical axis order
    (Section 2.3 defines a; the cube stencil evaluates it at the node)."""
    shape = _grid_shape(dim, n1, n2, n3)
    N = n1 * n2 * n3
    Tg = np.asarray(T, dtype=np.float64).reshape(shape)
    Gm = _metric_full(np.asarray(G, dtype=np.float64), dim, shape)
    nd = len(shape)
    D = [_central(Tg, nd - 1 - dd) for dd in range(dim)]
    out = np.empty((N, dim))
    for d in range(dim):
        acc = None
        for dp in range(dim):
            term = Gm[d][dp] * D[dp]
            acc = term if acc is None else acc + term
        out[:, d] = acc.reshape(N)
    return out


def cube_slot(off):
    """Neighbour slot 0..25 of a logical offset (o_0, o_1, o_2) in {-1,0,1}^3
    (o_2 = 0 in 2-D): 3-digit base-3 number of o + 1, axis 0 lowest, with the
    centre (13) left out."""
    b = (off[..., 0] + 1) + 3 * (off[..., 1] + 1) + 9 * (off[..., 2] + 1)
    return b - (b > 13)


def cube_couplings(dim, n1, n2, n3, G, T):
    """Upstream couplings of the 26-neighbour (cube) stencil: the backward
    characteristic of the node, p - t a with t = 1 / max_d |a_d| (unit logical
    spacing), leaves the node's 3x3x3 cube through the face of the dominant
    axis, and the transport value there is interpolated linearly on the
    simplex of the cube's Kuhn (Freudenthal) triangulation that contains it.
    With the axes sorted by r_d = |a_d| / max|a| (descending, ties to the lower
    axis) and u_d = -sign(a_d) the upstream step, the vertices are the partial
    sums u_(1) e_(1), + u_(2) e_(2), + u_(3) e_(3) with couplings
    r_(1) - r_(2), r_(2) - r_(3), r_(3) (2-D: r_(1) - r_(2), r_(2)).  An axis
    whose upstream neighbour lies outside the grid has its component of a set
    to 0 first (no inflow from outside, as a missing face contributes nothing
    in the face rule).

    Returns (slot, node, coupling), each [N, dim]; coupling 0 marks an unused
    vertex.  Nodes whose projected a vanishes get no vertex.

    parity: pinned by linear exactness along the characteristic on affine
    traveltimes (flat and anisotropic metrics, 2-D and 3-D), by reduction to
    the face rule for axis-aligned directions, and by the upwind-side,
    in-grid and vertex-count invariants (tests/test_oracle_cube.py).
    """
    N = n1 * n2 * n3
    a = node_directions(dim, n1, n2, n3, G, T)
    n = np.array([n1, n2, n3] if dim == 3 else [n1, n3], dtype=np.int64)
    stride = np.array([1, n1, n1 * n2] if dim == 3 else [1, n1], dtype=np.int64)
    ids = np.arange(N, dtype=np.int64)
    coord = (ids[:, None] // stride[None, :]) % n[None, :]
    up = np.where(a > 0.0, -1, np.where(a < 0.0, 1, 0)).astype(np.int64)
    inside = (coord + up >= 0) & (coord + up <= n[None, :] - 1)
    a = np.where(inside, a, 0.0)
    up = np.where(inside, up, 0)
    amax = np.max(np.abs(a), axis=1)
    live = amax > 0.0
    r = np.zeros_like(a)
    r[live] = np.abs(a[live]) / amax[live][:, None]
    order = np.argsort(-r, axis=1, kind="stable")
    rs = np.take_along_axis(r, order, axis=1)
    off = np.zeros((N, 3), dtype=np.int64)
    slot = np.zeros((N, dim), dtype=np.int64)
    node = np.zeros((N, dim), dtype=np.int64)
    coup = np.zeros((N, dim))
    rows = np.arange(N)
    for t in range(dim):
        ax = order[:, t]
        off[rows, ax] += up[rows, ax]
        slot[:, t] = cube_slot(off)
        node[:, t] = ids + off[:, :dim] @ stride
        coup[:, t] = rs[:, t] - rs[:, t + 1] if t + 1 < dim else rs[:, t]
    coup[~live] = 0.0
    return slot, node, coup


def _cube_rows(dim, n1, n2, n3, G, T, active):
    """Normalised rows of the cube stencil: couplings in ascending slot order,
    d = their sum in that order, w = c / d (eq. (discrete-row))."""
    slot, node, coup = cube_couplings(dim, n1, n2, n3, G, T)
    key = np.where(coup > 0.0, slot, 99)
    srt = np.argsort(key, axis=1, kind="stable")
    slot = np.take_along_axis(slot, srt, axis=1)
    node = np.take_along_axis(node, srt, axis=1)
    coup = np.take_along_axis(coup, srt, axis=1)
    N = coup.shape[0]
    dsum = np.zeros(N)
    for t in range(dim):
        dsum = dsum + coup[:, t]
    act = active & (dsum > 0.0)
    wslots = []
    for t in range(dim):
        w = np.zeros(N)
        m = act & (coup[:, t] > 0.0)
        w[m] = coup[m, t] / dsum[m]
        wslots.append((w, node[:, t]))
    return wslots


def assemble(dim, n1, n2, n3, G, T, s, src, rcv=None, rcv_w=None, identity_rows=None,
             stencil=6) -> OracleOperator:
    """Assemble W and c (Section 3.1 eq. (discrete-row), Section 3.2).

    identity_rows: further nodes whose rows are identity rows besides src
    (the source-seed rows of an off-grid point source, oracle.source); their
    calibration is then replaced by the seed derivative there.

    stencil: 6 for the face-based upwinding of Section 3.1; 26 for the cube
    stencil (cube_couplings), whose dependencies reach the edge and corner
    neighbours; both normalise the couplings and calibrate the right-hand
    side the same way.

    parity: pinned by the manufactured tangent test (first-order convergence to
    eq. (test-dT), Table 1), the flat-grid causal-order case, the 1-D closed
    form, the exact scaling identity and the reversal criterion; the cube
    stencil by the pins listed in cube_couplings.
    """
    shape = _grid_shape(dim, n1, n2, n3)
    N = n1 * n2 * n3
    T = np.asarray(T, dtype=np.float64).reshape(N)
    s = np.asarray(s, dtype=np.float64).reshape(N)
    if stencil not in (6, 26):
        raise ValueError("stencil must be 6 or 26")
    if stencil == 26:
        active = np.ones(N, dtype=bool)
        active[src] = False
        if identity_rows is not None:
            active[np.asarray(identity_rows, dtype=np.int64)] = False
        return _finish(dim, n1, n2, n3, T, s, src, rcv, rcv_w,
                       _cube_rows(dim, n1, n2, n3, G, T, active))
    a_faces, _ = face_coefficients(dim, n1, n2, n3, G, T)
    nd = len(shape)
    ids = np.arange(N, dtype=np.int64).reshape(shape)
    # slot order: axis 0 minus, axis 0 plus, axis 1 minus, ...
    slot_c, slot_j = [], []
    for d in range(dim):
        ax = nd - 1 - d
        n = shape[ax]
        a = a_faces[d]
        # minus face of node p (p = lo+1): coupling from p - e_d
        cm = np.zeros(shape)
        jm = np.full(shape, -1, dtype=np.int64)
        cm[_sl(nd, ax, slice(1, n))] = np.maximum(a, 0.0)
        jm[_sl(nd, ax, slice(1, n))] = ids[_sl(nd, ax, slice(0, n - 1))]
        # plus face of node p (p = lo): coupling from p + e_d
        cp = np.zeros(shape)
        jp = np.full(shape, -1, dtype=np.int64)
        cp[_sl(nd, ax, slice(0, n - 1))] = np.maximum(-a, 0.0)
        jp[_sl(nd, ax, slice(0, n - 1))] = ids[_sl(nd, ax, slice(1, n))]
        slot_c += [cm.reshape(N), cp.reshape(N)]
        slot_j += [jm.reshape(N), jp.reshape(N)]
    dsum = np.zeros(N)
    for cs in slot_c:
        dsum = dsum + cs
    active = dsum > 0.0
    active[src] = False
    if identity_rows is not None:
        active[np.asarray(identity_rows, dtype=np.int64)] = False
    wslots = []
    for cs, js in zip(slot_c, slot_j):
        w = np.zeros(N)
        m = active & (cs > 0.0)
        w[m] = cs[m] / dsum[m]
        wslots.append((w, js))
    return _finish(dim, n1, n2, n3, T, s, src, rcv, rcv_w, wslots)


def _finish(dim, n1, n2, n3, T, s, src, rcv, rcv_w, wslots) -> OracleOperator:
    """W from the per-slot weights, and c = (T - W T) / s with W T summed in
    slot order (Section 3.2)."""
    N = T.shape[0]
    rows, cols, vals = [], [], []
    for w, js in wslots:
        sel = np.nonzero(w > 0.0)[0]
        rows.append(sel)
        cols.append(js[sel])
        vals.append(w[sel])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    W = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    W.sum_duplicates()
    W.sort_indices()
    # l = A T = T - W T, slot order; c = l / s (Section 3.2)
    acc = np.zeros(N)
    for w, js in wslots:
        contrib = np.zeros(N)
        m = w > 0.0
        contrib[m] = w[m] * T[js[m]]
        acc = acc + contrib
    ell = T - acc
    c = ell / s
    if rcv is None:
        rcv = np.zeros(0, dtype=np.int64)
    return OracleOperator(dim=dim, n1=n1, n2=n2, n3=n3, W=W, c=c, src=int(src),
                          rcv=np.asarray(rcv, dtype=np.int64), T=T, s=s,
                          rcv_w=None if rcv_w is None else np.asarray(rcv_w, dtype=np.float64))


def assemble_workload(wl, alpha: int) -> OracleOperator:
    """Assemble the operator of source alpha of a workloads.Workload (its
    stencil attribute, 6 when absent)."""
    return assemble(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[alpha], wl.s, int(wl.src[alpha]),
                    wl.rcv, getattr(wl, "rcv_w", None), stencil=getattr(wl, "stencil", 6))
