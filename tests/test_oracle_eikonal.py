"""Pins of the first-arrival oracle (oracle/eikonal.py): the monotone
semi-Lagrangian update on the boundary-conforming grid (Section 2.1 defines
the state as the viscosity solution of |grad_x T| = s).

* segment_min / triangle_min equal a brute-force minimisation of
  T(y) + s |x - y| over the simplex (random cases, interior and boundary
  minima);
* a plane wave T = s k.x is a fixed point of the update at every interior
  node of a deformed grid (linear interpolation is exact for it and the
  backward ray meets one of the stencil's simplices), and the update never
  goes below it at boundary nodes;
* on a line of nodes the solution is the closed form T_i = T_{i-1} + s_i |x_i - x_{i-1}|;
* Jacobi and Gauss-Seidel reach the same fixed point on a deformed 3-D grid
  with a heterogeneous medium (the update is monotone);
* the update is monotone: raising neighbour values never lowers it;
* homogeneous medium, flat grid: the error against the exact distance falls
  under refinement.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W
from oracle import eikonal as E


def _brute_segment(xi, si, x1, t1, x2, t2):
    lam = np.linspace(0.0, 1.0, 20001)
    y = x1[None] + lam[:, None] * (x2 - x1)[None]
    f = (1 - lam) * t1 + lam * t2 + si * np.linalg.norm(xi[None] - y, axis=1)
    j = int(np.argmin(f))
    g = lambda l: (1 - l[0]) * t1 + l[0] * t2 + si * np.linalg.norm(xi - (x1 + l[0] * (x2 - x1)))
    r = minimize(g, [lam[j]], bounds=[(0.0, 1.0)], method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12})
    return min(f[j], float(r.fun))


def _brute_triangle(xi, si, xs, ts):
    best = np.inf
    n = 400
    for a in range(n + 1):
        l2 = np.arange(n + 1 - a) / n
        l1 = np.full_like(l2, a / n)
        l0 = 1 - l1 - l2
        y = l0[:, None] * xs[0] + l1[:, None] * xs[1] + l2[:, None] * xs[2]
        f = l0 * ts[0] + l1 * ts[1] + l2 * ts[2] + si * np.linalg.norm(xi[None] - y, axis=1)
        j = int(np.argmin(f))
        if f[j] < best:
            best, start = f[j], (l1[j], l2[j])

    def g(l):
        l0 = 1 - l[0] - l[1]
        y = l0 * xs[0] + l[0] * xs[1] + l[1] * xs[2]
        return l0 * ts[0] + l[0] * ts[1] + l[1] * ts[2] + si * np.linalg.norm(xi - y)
    cons = ({"type": "ineq", "fun": lambda l: 1 - l[0] - l[1]},)
    r = minimize(g, start, bounds=[(0, 1), (0, 1)], constraints=cons, method="SLSQP",
                 options={"ftol": 1e-15, "maxiter": 500})
    return min(best, float(r.fun)) if r.success else best


def test_segment_and_triangle_minima_against_brute_force():
    rng = np.random.default_rng(11)
    interior = 0
    for case in range(60):
        xi = rng.normal(size=3)
        xs = xi[None] + rng.normal(size=(3, 3)) + np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
        si = rng.uniform(0.3, 2.0)
        ts = rng.uniform(0.0, 1.5, size=3)
        got = float(E.segment_min(xi[None], np.array([si]), xs[0][None], ts[:1], xs[1][None], ts[1:2])[0])
        ref = _brute_segment(xi, si, xs[0], ts[0], xs[1], ts[1])
        assert got <= ref + 1e-12 and abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (case, got, ref)
        got = float(E.triangle_min(xi[None], np.array([si]), xs[0][None], ts[:1], xs[1][None], ts[1:2],
                                   xs[2][None], ts[2:3])[0])
        ref = _brute_triangle(xi, si, xs, ts)
        assert got <= ref + 1e-12 and abs(got - ref) <= 1e-8 * max(1.0, abs(ref)), (case, got, ref)
        # count cases whose minimum is inside the triangle (not on an edge)
        edges = min(float(E.segment_min(xi[None], np.array([si]), xs[a][None], ts[a:a + 1], xs[b][None],
                                        ts[b:b + 1])[0]) for a, b in ((0, 1), (0, 2), (1, 2)))
        interior += got < edges - 1e-9
    assert interior >= 5, interior


def test_plane_wave_is_a_fixed_point_on_a_deformed_grid():
    wl = W.smooth_3d(17, 15, 9, topo_amp=0.15, with_T=False)
    X = wl.X
    s = 0.4
    nb = E.neighbours(3, wl.n1, wl.n2, wl.n3)
    interior = np.all(nb >= 0, axis=(0, 1))
    rng = np.random.default_rng(12)
    for _ in range(5):
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        T = s * (X @ k) + 3.0
        F = E.update(3, nb, X, np.full(wl.N, s), T)
        assert np.max(np.abs(F[interior] - T[interior])) <= 1e-12 * np.abs(T).max()
        assert np.all(F >= T - 1e-12 * np.abs(T).max())


def test_line_of_nodes_closed_form():
    n1 = 40
    x = np.cumsum(np.random.default_rng(13).uniform(0.05, 0.2, n1))
    X = np.stack([x, np.zeros(n1)], axis=1)
    s = np.random.default_rng(14).uniform(0.2, 0.8, n1)
    src = 7
    T, it = E.solve(2, n1, 1, 1, X, s, src, radius=0)
    ref = np.zeros(n1)
    for i in range(src + 1, n1):
        ref[i] = ref[i - 1] + s[i] * (x[i] - x[i - 1])
    for i in range(src - 1, -1, -1):
        ref[i] = ref[i + 1] + s[i] * (x[i + 1] - x[i])
    assert np.max(np.abs(T - ref)) <= 1e-14 * ref.max()


def test_jacobi_and_gauss_seidel_reach_the_same_fixed_point():
    wl = W.smooth_3d(9, 8, 6, topo_amp=0.2, with_T=False)
    s = wl.s * (1.0 + 0.3 * np.sin(wl.X[:, 0] * 2.0) * np.cos(wl.X[:, 2] * 3.0))
    src = int(wl.node(3, 4, 0))
    Tj, itj = E.solve(3, wl.n1, wl.n2, wl.n3, wl.X, s, src, radius=1)
    Tg, itg = E.solve(3, wl.n1, wl.n2, wl.n3, wl.X, s, src, radius=1, order="gauss-seidel")
    assert np.all(np.isfinite(Tj))
    assert np.max(np.abs(Tj - Tg)) <= 2e-15 * Tj.max(), (itj, itg)
    # and it is a fixed point of the update off the seeds
    nb = E.neighbours(3, wl.n1, wl.n2, wl.n3)
    sn, _ = E.seeds(3, wl.n1, wl.n2, wl.n3, wl.X, s, src, 1)
    free = np.ones(wl.N, bool)
    free[sn] = False
    F = E.update(3, nb, wl.X, s, Tj)
    assert np.array_equal(np.minimum(Tj, F)[free], Tj[free])


def test_update_is_monotone():
    wl = W.smooth_3d(9, 8, 6, topo_amp=0.2, with_T=False)
    src = int(wl.node(4, 4, 0))
    T, _ = E.solve(3, wl.n1, wl.n2, wl.n3, wl.X, wl.s, src, radius=1)
    nb = E.neighbours(3, wl.n1, wl.n2, wl.n3)
    F0 = E.update(3, nb, wl.X, wl.s, T)
    rng = np.random.default_rng(15)
    for _ in range(5):
        F1 = E.update(3, nb, wl.X, wl.s, T + rng.uniform(0, 0.05, wl.N))
        assert np.all(F1 >= F0 - 1e-15)


def test_homogeneous_error_falls_under_refinement():
    errs = []
    for n in ((11, 11, 6), (21, 21, 11), (41, 41, 21)):
        wl = W.smooth_3d(*n, topo_amp=0.0, with_T=False)
        s = np.full(wl.N, 0.5)
        src = int(wl.node((n[0] - 1) // 2, (n[1] - 1) // 2, 0))
        T, _ = E.solve(3, wl.n1, wl.n2, wl.n3, wl.X, s, src, radius=1)
        ex = 0.5 * np.linalg.norm(wl.X - wl.X[src], axis=1)
        errs.append(np.max(np.abs(T - ex)) / ex.max())
    print("homogeneous max errors", errs)
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]
