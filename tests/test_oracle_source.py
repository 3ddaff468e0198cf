"""Pins of the off-grid point-source oracle (oracle/source.py): the
source-seed rows of Section 3.1, their right-hand side from the
differentiated source treatment (Section 3.2) and the direct data term
D_alpha of eq. (source-jacobian) / eq. (source-transpose).

* A source on a node with seed radius 0 is the on-grid operator (identity
  source row, c_src = 0, D = 0): the same J and J^T.
* Scaling identity: every seed time and every direct time is homogeneous of
  degree one in s and c = (A T)/s off the seeds, so J s equals the predicted
  data exactly (up to rounding).
* The seed rows of C and the rows of D equal central finite differences of
  the straight-ray formulas they differentiate.
* Transpose pairing <J p, y> = <p, J^T y> with direct receivers present.
* Homogeneous medium, flat grid, linear ds: the transported perturbation
  converges to the exact eq. (test-dT) at first order under refinement.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import source as PS
from oracle.assembly import assemble


def _case(n=(21, 21, 11), xi=(7.3, 9.6, 0.0), rho=1.5, topo=0.1):
    wl = W.smooth_3d(*n, topo_amp=topo, with_T=False)
    xi = np.array(xi)
    W.eikonal_point(wl, xi[None, :], rho)
    # surface receivers: the lattice, one node inside the seed region (direct)
    # and one interpolating receiver next to the source (direct)
    L = PS.node_logical(3, wl.n1, wl.n2, wl.n3)
    near = int(np.argmin(np.sum((L - (xi + np.array([1.0, 0.0, 0.0]))) ** 2, axis=1)))
    nodes = np.concatenate([wl.rcv, [near]])
    R = nodes.size + 1
    rcv = np.zeros((R, 2), dtype=np.int64)
    w = np.zeros((R, 2))
    rcv[:-1, 0] = nodes
    rcv[:-1, 1] = nodes
    w[:-1, 0] = 1.0
    i0 = int(np.floor(xi[0])) - 1
    j0 = int(np.round(xi[1]))
    rcv[-1] = [i0 + wl.n1 * j0, i0 + 1 + wl.n1 * j0]
    w[-1] = [0.4, 0.6]
    return wl, xi, rho, rcv, w


def test_source_on_a_node_with_no_seed_region_is_the_on_grid_operator():
    wl, _, _, rcv, w = _case()
    src = int(wl.rcv[7])          # a surface node
    L = PS.node_logical(3, wl.n1, wl.n2, wl.n3)
    xi = L[src]
    W.eikonal_point(wl, xi[None, :], 0.0)
    T = wl.T[0]
    assert T[src] == 0.0
    pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, T, wl.s, xi, 0.0, rcv, w)
    # the receiver on the source node is "direct" with a zero-length ray: its
    # row of D is zero, as the on-grid source row gives dT = 0 there
    assert list(pso.seeds) == [src] and np.count_nonzero(pso.D.data) == 0
    op = assemble(3, wl.n1, wl.n2, wl.n3, wl.G, T, wl.s, src, rcv, w)
    rng = np.random.default_rng(1)
    ds = rng.standard_normal(wl.N)
    y = rng.standard_normal(rcv.shape[0])
    ref = O.apply_J(op, ds, "receivers", "superlu")
    got = PS.apply_J(pso, ds)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())
    assert np.array_equal(PS.apply_J(pso, ds, "nodes"), O.apply_J(op, ds, "nodes", "superlu"))
    g_ref = O.apply_JT(op, y, "receivers", "superlu")
    assert np.allclose(PS.apply_JT(pso, y), g_ref, rtol=1e-12, atol=1e-14 * np.abs(g_ref).max())


def test_scaling_identity_with_seed_rows_and_direct_receivers():
    wl, xi, rho, rcv, w = _case()
    T = wl.T[0]
    pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, T, wl.s, xi, rho, rcv, w)
    assert pso.seeds.size > 1 and pso.direct.size >= 2
    # the seed times are the straight-ray formula of the generator
    seeds, Ts, _, _ = PS.seed_traveltime(3, wl.n1, wl.n2, wl.n3, wl.X, wl.s, xi, rho)
    assert np.array_equal(seeds, pso.seeds)
    assert np.allclose(T[seeds], Ts, rtol=1e-14, atol=0)
    d = PS.predicted_data(pso, 3, wl.n1, wl.n2, wl.n3, wl.X, T, wl.s, xi, rcv, w)
    Js = PS.apply_J(pso, wl.s)
    assert np.linalg.norm(Js - d) <= 1e-13 * np.linalg.norm(d)
    assert np.linalg.norm(PS.apply_J(pso, wl.s, "nodes") - T) <= 1e-13 * np.linalg.norm(T)


def test_seed_rows_and_direct_rows_are_derivatives_of_the_straight_ray_times():
    wl, xi, rho, rcv, w = _case()
    T = wl.T[0]
    pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, T, wl.s, xi, rho, rcv, w)
    rng = np.random.default_rng(2)
    ds = wl.s * rng.uniform(-1, 1, wl.N)
    eps = 1e-6
    sp_, sm = wl.s + eps * ds, wl.s - eps * ds
    _, Tp, _, _ = PS.seed_traveltime(3, wl.n1, wl.n2, wl.n3, wl.X, sp_, xi, rho)
    _, Tm, _, _ = PS.seed_traveltime(3, wl.n1, wl.n2, wl.n3, wl.X, sm, xi, rho)
    q = pso.C @ ds
    fd = (Tp - Tm) / (2 * eps)
    assert np.allclose(q[pso.seeds], fd, rtol=1e-8, atol=1e-12 * np.abs(fd).max())
    dp = PS.predicted_data(pso, 3, wl.n1, wl.n2, wl.n3, wl.X, T, sp_, xi, rcv, w)
    dm = PS.predicted_data(pso, 3, wl.n1, wl.n2, wl.n3, wl.X, T, sm, xi, rcv, w)
    fd = (dp - dm)[pso.direct] / (2 * eps)
    assert np.allclose((pso.D @ ds)[pso.direct], fd, rtol=1e-8, atol=1e-12 * np.abs(fd).max())


def test_transpose_pairing_with_direct_term():
    wl, xi, rho, rcv, w = _case()
    pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, wl.T[0], wl.s, xi, rho, rcv, w)
    rng = np.random.default_rng(3)
    for _ in range(3):
        p = rng.standard_normal(wl.N)
        y = rng.standard_normal(rcv.shape[0])
        a, b = PS.apply_J(pso, p) @ y, p @ PS.apply_JT(pso, y)
        assert abs(a - b) <= 1e-13 * max(abs(a), abs(b))
        yn = rng.standard_normal(wl.N)
        a, b = PS.apply_J(pso, p, "nodes") @ yn, p @ PS.apply_JT(pso, yn, "nodes")
        assert abs(a - b) <= 1e-13 * max(abs(a), abs(b))


def test_off_grid_source_first_order_against_the_exact_tangent():
    """eq. (test-dT): in a homogeneous medium with a linear slowness
    perturbation, dT_ex(x) = |x - x_s|/2 (ds(x_s) + ds(x)).  On a flat grid
    with the source between nodes, the transported perturbation converges to
    it at first order."""
    errs = []
    for n in ((21, 21, 11), (41, 41, 21), (81, 81, 41)):
        wl = W.smooth_3d(*n, topo_amp=0.0, with_T=False)
        wl.s = np.full(wl.N, 1.0 / 3.0)
        xi = np.array([0.3 * (n[0] - 1) + 0.37, 0.55 * (n[1] - 1) + 0.21, 0.0])
        X = wl.X
        cn, phi = PS.cell_weights(3, wl.n1, wl.n2, wl.n3, xi)
        xs = np.sum(phi[:, None] * X[cn], axis=0)
        # the exact traveltime of the homogeneous medium (as in Section 5.1),
        # which the straight-ray seed formula reproduces on the seeds
        T = wl.s * np.sqrt(np.sum((X - xs[None, :]) ** 2, axis=1))
        pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, T, wl.s, xi, 1.5, wl.rcv)
        a = np.array([0.02, 0.04, -0.03])
        ds = wl.s * (a[0] * X[:, 0] + a[1] * X[:, 1] + a[2] * X[:, 2]) / 4.0
        dss = float(np.sum(phi * ds[cn]))
        r = np.sqrt(np.sum((X - xs[None, :]) ** 2, axis=1))
        ex = 0.5 * r * (dss + ds)
        got = PS.apply_J(pso, ds, "nodes")
        errs.append(np.linalg.norm(got - ex) / np.linalg.norm(ex))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[2] < errs[1] < errs[0]
    assert np.all(order > 0.8), (errs, order)
