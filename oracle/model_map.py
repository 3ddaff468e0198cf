"""Cell-velocity model map M_alpha of Section 4.4 (eq. (source-jacobian)):
the oracle's plain version (test infrastructure; only tests, smoke and the
benchmark's CPU leg use this package).

The model is one velocity per cell of the logical grid (hexahedra between
nodes, quadrilaterals in 2-D).  A node's slowness is the reciprocal of the
mean velocity of the cells that share it.  M is the derivative of that map
at the given velocities, written out entry by entry; parity pins:
finite differences of cell_slowness, the constant-velocity closed form and
the number of cells per node (tests/test_oracle_model_map.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _axes(dim, n1, n2, n3):
    return (n1, n2, n3) if dim == 3 else (n1, n3, 1)


def _cells_of_node(i, n):
    """Cell indices along one axis that touch node index i (n nodes)."""
    if n == 1:
        return [0]
    return [c for c in (i - 1, i) if 0 <= c <= n - 2]


def cell_count(dim, n1, n2, n3) -> int:
    a = _axes(dim, n1, n2, n3)
    return int(np.prod([max(m - 1, 1) for m in a]))


def _node_cells(dim, n1, n2, n3):
    """For every node, in node order, the ids of the cells that share it."""
    a0, a1, a2 = _axes(dim, n1, n2, n3)
    c0, c1 = max(a0 - 1, 1), max(a1 - 1, 1)
    out = []
    for k in range(a2):
        for j in range(a1):
            for i in range(a0):
                out.append([ci + c0 * (cj + c1 * ck) for ck in _cells_of_node(k, a2)
                            for cj in _cells_of_node(j, a1) for ci in _cells_of_node(i, a0)])
    return out


def cell_slowness(dim, n1, n2, n3, v) -> np.ndarray:
    """Nodal slowness s_p = 1 / mean(v_c over the cells c that share node p)."""
    v = np.asarray(v, dtype=np.float64)
    return np.array([1.0 / np.mean(v[cs]) for cs in _node_cells(dim, n1, n2, n3)])


def model_map_matrix(dim, n1, n2, n3, v) -> sp.csr_matrix:
    """M = d s / d v: for node p with n_p cells and mean velocity vbar_p,
    M[p, c] = -1 / (n_p vbar_p^2) for each of its cells c."""
    v = np.asarray(v, dtype=np.float64)
    rows, cols, vals = [], [], []
    for p, cs in enumerate(_node_cells(dim, n1, n2, n3)):
        vbar = np.mean(v[cs])
        for c in cs:
            rows.append(p)
            cols.append(c)
            vals.append(-1.0 / (len(cs) * vbar * vbar))
    N = int(np.prod(_axes(dim, n1, n2, n3)))
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, cell_count(dim, n1, n2, n3)))
