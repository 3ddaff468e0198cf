"""Pins of the 26-neighbour (cube) stencil of the oracle (no GPU).

The cube stencil takes the transport value at the point where the node's
backward characteristic (direction -a, a = G grad_xi T, Section 2.3) leaves
the node's 3x3x3 cube, interpolated linearly on the Kuhn simplex that holds
that point; rows are normalised and calibrated as in Sections 3.1-3.2.  The
pins do not restate the construction:

* linear exactness along the characteristic: on an affine traveltime the
  direction a is known in closed form (M k for a constant metric M and
  T = k.xi), and for every affine field L the row gives
  L_p - (W L)_p = (grad L . a) / max|a| exactly (interpolation is exact for
  affine functions), for flat, anisotropic and sheared metrics, 2-D and 3-D,
  random signs and tied components;
* an axis-aligned direction reduces the row to the face rule's row;
* invariants on a deformed grid: at most dim dependencies per row, each in the
  node's 3x3x3 cube, inside the grid and on the upstream side of a; weights
  positive and summing to 1; edge and corner neighbours occur;
* the scaling identity J s = T of the calibration (Section 3.2);
* planted mistakes (swapped couplings, a vertex mirrored to the downstream
  side, a wrong cross-metric entry) each fail the exactness pin.
"""
import numpy as np
import pytest

import oracle as O
import oracle.assembly as OA
import workloads as W


def _flat(dim, n, M, k, x0=None):
    """Flat unit grid, constant metric M (dim x dim), affine T = k . (xi - x0)."""
    if dim == 3:
        n1, n2, n3 = n
        G = np.tile([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]], (n1 * n2 * n3, 1))
        xi = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
        xi = xi.transpose(2, 1, 0, 3).reshape(-1, 3).astype(float)
    else:
        n1, n3 = n
        n2 = 1
        G = np.tile([M[0, 0], M[1, 1], M[0, 1]], (n1 * n3, 1))
        xi = np.stack(np.meshgrid(np.arange(n1), np.arange(n3), indexing="ij"), -1)
        xi = xi.transpose(1, 0, 2).reshape(-1, 2).astype(float)
    x0 = np.zeros(dim) if x0 is None else np.asarray(x0, float)
    T = (xi - x0) @ k
    return n1, n2, n3, G, T, xi


def _interior(xi, n):
    n = np.asarray(n)
    return np.all((xi >= 1) & (xi <= n - 2), axis=1)


CASES = [
    (3, (7, 6, 5), np.eye(3), [0.9, -0.4, 0.25]),
    (3, (7, 6, 5), np.diag([1.3, 0.7, 2.1]), [-0.3, 0.5, 0.8]),
    (3, (6, 7, 6), np.array([[1.2, 0.3, -0.2], [0.3, 0.9, 0.1], [-0.2, 0.1, 1.5]]), [0.2, 0.6, -0.7]),
    (3, (6, 6, 6), np.eye(3), [0.5, -0.5, 0.5]),          # every component tied
    (3, (6, 6, 6), np.eye(3), [0.5, 0.5, -0.2]),          # two tied
    (3, (6, 6, 6), np.eye(3), [0.0, 0.7, -0.3]),          # one zero component
    (2, (9, 7), np.eye(2), [0.6, -0.35]),
    (2, (9, 7), np.array([[1.1, -0.4], [-0.4, 0.8]]), [-0.5, -0.9]),
    (2, (8, 8), np.eye(2), [0.4, 0.4]),
]


@pytest.mark.parametrize("dim,n,M,k", CASES)
def test_linear_exactness_along_the_characteristic(dim, n, M, k):
    k = np.asarray(k, float)
    n1, n2, n3, G, T, xi = _flat(dim, n, M, k, x0=np.full(dim, 2.0))
    a = M @ k
    op = OA.assemble(dim, n1, n2, n3, G, T, np.ones(T.size), src=0, stencil=26)
    inner = _interior(xi, n)
    inner[0] = False
    rng = np.random.default_rng(71)
    for _ in range(4):
        g = rng.normal(size=dim)
        L = xi @ g
        lhs = L - op.W @ L
        rhs = (g @ a) / np.max(np.abs(a))
        assert np.max(np.abs(lhs[inner] - rhs)) <= 1e-13 * max(1.0, np.abs(L).max())
    # every interior row is an interpolation: weights sum to 1
    rs = np.asarray(op.W.sum(axis=1)).ravel()
    assert np.max(np.abs(rs[inner] - 1.0)) <= 4e-16


def test_axis_aligned_direction_reduces_to_the_face_rule():
    for dim, n, M, k in [(3, (6, 5, 4), np.diag([1.0, 2.0, 0.5]), [0.7, 0.0, 0.0]),
                         (3, (6, 5, 4), np.eye(3), [0.0, -0.4, 0.0]),
                         (3, (5, 5, 6), np.diag([0.8, 1.1, 1.7]), [0.0, 0.0, 0.9]),
                         (2, (7, 6), np.diag([1.4, 0.6]), [0.0, -0.8])]:
        k = np.asarray(k, float)
        n1, n2, n3, G, T, xi = _flat(dim, n, M, k, x0=np.full(dim, 2.0))
        face = OA.assemble(dim, n1, n2, n3, G, T, np.ones(T.size), src=0, stencil=6)
        cube = OA.assemble(dim, n1, n2, n3, G, T, np.ones(T.size), src=0, stencil=26)
        assert (face.W != cube.W).nnz == 0
        assert np.array_equal(face.c, cube.c)


def _deformed():
    wl = W.smooth_3d(13, 11, 9, topo_amp=0.2)
    wl.stencil = 26
    return wl


def test_invariants_on_a_deformed_grid():
    wl = _deformed()
    op = OA.assemble_workload(wl, 0)
    Wc = op.W.tocsr()
    a = OA.node_directions(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[0])
    n = np.array([wl.n1, wl.n2, wl.n3])
    ids = np.arange(wl.N)
    xi = np.stack([ids % wl.n1, (ids // wl.n1) % wl.n2, ids // (wl.n1 * wl.n2)], 1)
    kinds = set()
    for i in range(wl.N):
        lo, hi = Wc.indptr[i], Wc.indptr[i + 1]
        if hi == lo:
            continue
        assert hi - lo <= 3
        w = Wc.data[lo:hi]
        assert np.all(w > 0) and abs(w.sum() - 1.0) <= 4e-16
        for j in Wc.indices[lo:hi]:
            off = xi[j] - xi[i]
            assert np.all(np.abs(off) <= 1) and np.any(off != 0)
            assert np.all((xi[j] >= 0) & (xi[j] < n))
            assert np.all(off * a[i] <= 0.0)            # never downstream of a
            kinds.add(int(np.count_nonzero(off)))
    assert kinds == {1, 2, 3}                           # face, edge and corner neighbours
    assert op.W.nnz > wl.N                              # more than one dependency on average


def test_scaling_identity():
    wl = _deformed()
    op = OA.assemble_workload(wl, 0)
    x = O.superlu_solve(op, op.c * wl.s)
    assert np.max(np.abs(x - wl.T[0])) <= 1e-12 * wl.T[0].max()


def test_deformed_2d_invariants_and_scaling():
    wl = W.grids.deformed_2d(41, 21, 5, 0.3, 2, S=1, B=1, R=4, name="2-D 41x21")
    W.eikonal(wl)
    wl.stencil = 26
    op = OA.assemble_workload(wl, 0)
    rs = np.asarray(op.W.sum(axis=1)).ravel()
    nz = np.diff(op.W.indptr) > 0
    assert np.max(np.abs(rs[nz] - 1.0)) <= 4e-16 and np.max(np.diff(op.W.indptr)) <= 2
    x = O.superlu_solve(op, op.c * wl.s)
    assert np.max(np.abs(x - wl.T[0])) <= 1e-12 * wl.T[0].max()


# ---- planted mistakes -------------------------------------------------------

def _mutant(kind):
    orig = OA.cube_couplings

    def mutated(dim, n1, n2, n3, G, T):
        if kind == "wrong_cross_metric":
            Gc = np.array(G, dtype=float, copy=True)
            if dim == 3:
                Gc[:, [3, 4]] = Gc[:, [4, 3]]
            else:
                Gc[:, 2] = -Gc[:, 2]
            return orig(dim, n1, n2, n3, Gc, T)
        slot, node, coup = orig(dim, n1, n2, n3, G, T)
        if kind == "swapped_couplings":
            coup = coup[:, ::-1].copy()
        elif kind == "mirrored_vertex":
            ids = np.arange(node.shape[0])
            mir = 2 * ids - node[:, -1]
            ok = (mir >= 0) & (mir < node.shape[0])
            node = node.copy()
            node[ok, -1] = mir[ok]
        return slot, node, coup
    return mutated, orig


@pytest.mark.parametrize("kind", ["swapped_couplings", "mirrored_vertex", "wrong_cross_metric"])
def test_planted_mistakes_fail_a_pin(kind, monkeypatch):
    mutated, orig = _mutant(kind)
    monkeypatch.setattr(OA, "cube_couplings", mutated)
    failed = False
    for dim, n, M, k in CASES[2:3] + CASES[7:8]:
        k = np.asarray(k, float)
        n1, n2, n3, G, T, xi = _flat(dim, n, M, k, x0=np.full(dim, 2.0))
        a = M @ k
        op = OA.assemble(dim, n1, n2, n3, G, T, np.ones(T.size), src=0, stencil=26)
        inner = _interior(xi, n)
        inner[0] = False
        g = np.random.default_rng(5).normal(size=dim)
        L = xi @ g
        err = np.max(np.abs((L - op.W @ L)[inner] - (g @ a) / np.max(np.abs(a))))
        failed |= err > 1e-13 * max(1.0, np.abs(L).max())
    assert failed
