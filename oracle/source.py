"""Off-grid point source, source-seed rows and the direct data term
(oracle; test infrastructure; shares no code with the library).

Section 3.1 treats source-seed rows apart from the generic interior rows,
Section 3.2 takes their right-hand side from the differentiated source
treatment, and eq. (source-jacobian) keeps a direct term D_alpha for source
configurations whose differentiated source treatment feeds receiver values
directly.  The paper gives no formulas; the reading written out here:

  * the source sits at logical coordinates xi_s inside the grid; its cell's
    2^dim corners k carry multilinear weights phi_k(xi_s), so
    s_src = sum_k phi_k s_k and x_src = sum_k phi_k X_k;
  * the seed region is every node p with max_d |i_d(p) - xi_s,d| <= rho; its
    traveltime is the straight-ray time T_p = (s_src + s_p)/2 |X_p - x_src|,
    its rows of A are identity rows, and their right-hand side is the
    derivative of that time: q_p = |X_p - x_src|/2 (sum_k phi_k ds_k + ds_p)
    (a row of C instead of the diagonal c_p of Section 3.2);
  * a receiver whose position (the weights of its entries applied to the
    logical coordinates) lies in the seed region takes the straight-ray time
    directly, d_r = (s_src + s_r)/2 |x_r - x_src| with s_r, x_r interpolated by
    the receiver's own weights; its row of P is zero and its row of D_alpha is
    |x_r - x_src|/2 (sum_k phi_k ds_k + sum_e w_e ds_e);
  * then J = P A^{-1} C + D and J^T = C^T A^{-T} P^T + D^T (eq. (source-jacobian),
    eq. (source-transpose)), every matrix explicit.

parity: pinned by the reduction to the on-grid operator (a source on a node
with rho = 0), the exact scaling identity J s = d(s) (every seed time and
direct time is homogeneous of degree one in s), central finite differences
of the seed and direct formulas, and the transpose pairing with D
(tests/test_oracle_source.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import OracleOperator, assemble


def _axes(dim, n1, n2, n3):
    return (n1, n2, n3) if dim == 3 else (n1, n3)


def node_logical(dim, n1, n2, n3):
    """Logical coordinates [N][dim] of every node (axis 0 fastest)."""
    ax = _axes(dim, n1, n2, n3)
    grids = np.meshgrid(*[np.arange(a, dtype=np.float64) for a in ax], indexing="ij")
    N = int(np.prod(ax))
    # node id = i + n1 (j + n2 k): axis 0 fastest
    out = np.empty((N, dim))
    for d in range(dim):
        out[:, d] = np.transpose(grids[d], list(range(dim))[::-1]).reshape(N)
    return out


def cell_weights(dim, n1, n2, n3, xi):
    """The 2^dim corners of the cell holding logical point xi and their
    multilinear weights (a node on a cell face or corner gets weight 1 there)."""
    ax = _axes(dim, n1, n2, n3)
    xi = np.asarray(xi, dtype=np.float64)
    base = [int(min(max(np.floor(xi[d]), 0), max(ax[d] - 2, 0))) for d in range(dim)]
    t = [xi[d] - base[d] for d in range(dim)]
    nodes, w = [], []
    for corner in range(1 << dim):
        idx, wt = [], 1.0
        for d in range(dim):
            up = (corner >> d) & 1
            idx.append(base[d] + up if ax[d] > 1 else base[d])
            wt *= t[d] if up else 1.0 - t[d]
        stride, nid = 1, 0
        for d in range(dim):
            nid += idx[d] * stride
            stride *= ax[d]
        nodes.append(nid)
        w.append(wt)
    return np.array(nodes, dtype=np.int64), np.array(w)


def seed_nodes(dim, n1, n2, n3, xi, rho):
    """Nodes p with max_d |i_d(p) - xi_d| <= rho, ascending."""
    L = node_logical(dim, n1, n2, n3)
    m = np.all(np.abs(L - np.asarray(xi, dtype=np.float64)[None, :]) <= rho, axis=1)
    return np.nonzero(m)[0].astype(np.int64)


def seed_traveltime(dim, n1, n2, n3, X, s, xi, rho):
    """(seed nodes, their straight-ray times, s_src, x_src)."""
    cn, phi = cell_weights(dim, n1, n2, n3, xi)
    s_src = float(np.sum(phi * s[cn]))
    x_src = np.sum(phi[:, None] * X[cn], axis=0)
    seeds = seed_nodes(dim, n1, n2, n3, xi, rho)
    r = np.sqrt(np.sum((X[seeds] - x_src[None, :]) ** 2, axis=1))
    return seeds, 0.5 * (s_src + s[seeds]) * r, s_src, x_src


@dataclass
class PointSourceOperator:
    """A = I - W with identity seed rows, the explicit C, P (zero rows for
    direct receivers) and D, for one off-grid source."""
    op: OracleOperator
    C: sp.csr_matrix
    P: sp.csr_matrix
    D: sp.csr_matrix
    seeds: np.ndarray
    direct: np.ndarray     # receiver indices taken directly

    @property
    def N(self):
        return self.op.N


def assemble_point_source(dim, n1, n2, n3, G, X, T, s, xi, rho, rcv, rcv_w=None, stencil=6) -> PointSourceOperator:
    N = n1 * n2 * n3
    s = np.asarray(s, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(N, dim)
    cn, phi = cell_weights(dim, n1, n2, n3, xi)
    s_src = float(np.sum(phi * s[cn]))
    x_src = np.sum(phi[:, None] * X[cn], axis=0)
    seeds = seed_nodes(dim, n1, n2, n3, xi, rho)
    # W with identity rows at the seeds (the src argument is one of them)
    op = assemble(dim, n1, n2, n3, G, T, s, int(seeds[0]), None, None, identity_rows=seeds, stencil=stencil)
    # C: the Section 3.2 diagonal off the seeds, the seed derivative on them
    c = op.c.copy()
    c[seeds] = 0.0
    rows, cols, vals = list(np.arange(N)), list(np.arange(N)), list(c)
    for p in seeds:
        half_r = 0.5 * float(np.sqrt(np.sum((X[p] - x_src) ** 2)))
        rows += [int(p)] * (len(cn) + 1)
        cols += list(cn) + [int(p)]
        vals += list(half_r * phi) + [half_r]
    C = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    C.sum_duplicates()
    # receivers: entries [R][K] (or [R]) with weights; direct if inside the seed region
    nodes = np.asarray(rcv, dtype=np.int64)
    if nodes.ndim == 1:
        nodes = nodes[:, None]
    w = np.ones(nodes.shape) if rcv_w is None else np.asarray(rcv_w, dtype=np.float64)
    R, K = nodes.shape
    L = node_logical(dim, n1, n2, n3)
    xi_r = np.einsum("rk,rkd->rd", w, L[nodes])
    direct = np.nonzero(np.all(np.abs(xi_r - np.asarray(xi)[None, :]) <= rho, axis=1))[0]
    is_direct = np.zeros(R, bool)
    is_direct[direct] = True
    prow, pcol, pval, drow, dcol, dval = [], [], [], [], [], []
    for r in range(R):
        if is_direct[r]:
            x_r = np.sum(w[r][:, None] * X[nodes[r]], axis=0)
            half_r = 0.5 * float(np.sqrt(np.sum((x_r - x_src) ** 2)))
            drow += [r] * (len(cn) + K)
            dcol += list(cn) + list(nodes[r])
            dval += list(half_r * phi) + list(half_r * w[r])
        else:
            prow += [r] * K
            pcol += list(nodes[r])
            pval += list(w[r])
    P = sp.csr_matrix((pval, (prow, pcol)), shape=(R, N))
    D = sp.csr_matrix((dval, (drow, dcol)), shape=(R, N))
    P.sum_duplicates()
    D.sum_duplicates()
    return PointSourceOperator(op=op, C=C.tocsr(), P=P, D=D, seeds=seeds, direct=direct)


def predicted_data(pso: PointSourceOperator, dim, n1, n2, n3, X, T, s, xi, rcv, rcv_w=None):
    """The data the point-source forward model predicts: P T at ordinary
    receivers, the straight-ray time at direct ones."""
    N = n1 * n2 * n3
    X = np.asarray(X, dtype=np.float64).reshape(N, dim)
    cn, phi = cell_weights(dim, n1, n2, n3, xi)
    s_src = float(np.sum(phi * s[cn]))
    x_src = np.sum(phi[:, None] * X[cn], axis=0)
    nodes = np.asarray(rcv, dtype=np.int64)
    if nodes.ndim == 1:
        nodes = nodes[:, None]
    w = np.ones(nodes.shape) if rcv_w is None else np.asarray(rcv_w, dtype=np.float64)
    d = pso.P @ T
    for r in pso.direct:
        x_r = np.sum(w[r][:, None] * X[nodes[r]], axis=0)
        s_r = float(np.sum(w[r] * s[nodes[r]]))
        d[r] = 0.5 * (s_src + s_r) * float(np.sqrt(np.sum((x_r - x_src) ** 2)))
    return d


def _lu(pso):
    if getattr(pso, "_lu", None) is None:
        pso._lu = spla.splu(pso.op.A().tocsc())
    return pso._lu


def apply_J(pso: PointSourceOperator, ds, out="receivers"):
    """J ds = P A^{-1} C ds + D ds (receivers) or A^{-1} C ds (nodes)."""
    ds = np.asarray(ds, dtype=np.float64)
    x = _lu(pso).solve(pso.C @ ds)
    if out == "nodes":
        return x
    return pso.P @ x + pso.D @ ds


def apply_JT(pso: PointSourceOperator, y, w_mode="receivers"):
    """J^T y = C^T A^{-T} P^T y + D^T y (receiver data) or C^T A^{-T} y (nodal)."""
    y = np.asarray(y, dtype=np.float64)
    if w_mode == "nodes":
        return pso.C.T @ _lu(pso).solve(y, trans="T")
    lam = _lu(pso).solve(pso.P.T @ y, trans="T")
    return pso.C.T @ lam + pso.D.T @ y
