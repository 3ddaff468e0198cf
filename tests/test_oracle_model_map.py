"""The cell-velocity model map M_alpha of Section 4.4 in the oracle (no GPU).

Pins of oracle.model_map against the mathematics, not against itself:
* M (the derivative written out) equals central finite differences of the
  nonlinear map v -> s (cell_slowness) on small 2-D and 3-D grids;
* a constant velocity v0 gives s = 1/v0 everywhere and rows of M summing
  to -1/v0^2;
* a node has 1 (corner), 2 (edge), 4 (face) or 8 (interior) cells in 3-D,
  1, 2 or 4 in 2-D.
"""
import numpy as np
import pytest

from oracle.model_map import cell_count, cell_slowness, model_map_matrix

GRIDS = [(2, 6, 1, 5), (3, 5, 4, 3)]


@pytest.mark.parametrize("g", GRIDS, ids=["2d", "3d"])
def test_matrix_is_the_derivative(g):
    dim, n1, n2, n3 = g
    Nc = cell_count(dim, n1, n2, n3)
    v = np.random.default_rng(11).uniform(1.5, 3.5, Nc)
    M = model_map_matrix(dim, n1, n2, n3, v).toarray()
    fd = np.zeros_like(M)
    for c in range(Nc):
        h = 1e-5 * v[c]
        vp, vm = v.copy(), v.copy()
        vp[c] += h
        vm[c] -= h
        fd[:, c] = (cell_slowness(dim, n1, n2, n3, vp) - cell_slowness(dim, n1, n2, n3, vm)) / (2 * h)
    assert np.max(np.abs(M - fd)) <= 1e-8 * np.max(np.abs(M))


@pytest.mark.parametrize("g", GRIDS, ids=["2d", "3d"])
def test_constant_velocity(g):
    dim, n1, n2, n3 = g
    v0 = 2.5
    v = np.full(cell_count(dim, n1, n2, n3), v0)
    assert np.allclose(cell_slowness(dim, n1, n2, n3, v), 1.0 / v0, rtol=0, atol=1e-15)
    M = model_map_matrix(dim, n1, n2, n3, v)
    assert np.allclose(np.asarray(M.sum(axis=1)).ravel(), -1.0 / v0 ** 2, rtol=1e-14, atol=0)


def test_cells_per_node():
    M3 = model_map_matrix(3, 5, 4, 3, np.ones(cell_count(3, 5, 4, 3)))
    nnz = np.diff(M3.indptr).reshape(3, 4, 5)
    assert nnz[0, 0, 0] == 1 and nnz[1, 0, 0] == 2 and nnz[1, 1, 0] == 4 and nnz[1, 1, 1] == 8
    assert sorted(set(nnz.ravel())) == [1, 2, 4, 8]
    M2 = model_map_matrix(2, 6, 1, 5, np.ones(cell_count(2, 6, 1, 5)))
    assert sorted(set(np.diff(M2.indptr))) == [1, 2, 4]
