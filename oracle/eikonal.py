"""First-arrival traveltimes by a monotone semi-Lagrangian update on the
boundary-conforming grid (oracle; test infrastructure; shares no code with the
library).

Section 2.1 defines the state: T is the viscosity solution of the isotropic
eikonal equation |grad_x T| = s with T = 0 at the source; the paper's own
solver (a factored full-metric formulation) is only cited.  The discrete
problem written out here:

  * the stencil of node i is its face neighbours (one logical step along each
    axis, inside the grid); its simplices are the neighbours themselves, the
    segments joining two neighbours on different axes and, in 3-D, the
    triangles with one neighbour on each axis;
  * the update is T_i = min over those simplices S, min over points y of S, of
    T_S(y) + s_i |x_i - y|, with T_S the linear interpolation of the vertex
    values over S and x the physical node positions;
  * seed nodes (max-norm logical distance <= r from the source node) keep the
    straight-ray time (s_src + s_p)/2 |x_p - x_src|, 0 at the source;
  * the solution is the fixed point reached from T = +inf off the seeds.

The update is a minimum of functions that are non-decreasing in the
neighbour values (each is a convex combination of them plus a fixed cost), so
it is monotone: from T = +inf every iteration decreases T towards the largest
fixed point, whatever the order in which nodes are updated.  The inner
minimum over a simplex is convex in the barycentric coordinates, so it is the
least of the stationary points that fall inside the simplex and the minima
over its faces; those stationary points have closed forms (segment_min,
triangle_min).

parity: pinned by brute-force minimisation over the simplex (random cases),
plane waves reproduced exactly, the 1-D closed form, Jacobi and Gauss-Seidel
reaching the same fixed point, and first-order convergence to the exact
distance in a homogeneous medium (tests/test_oracle_eikonal.py).
"""
from __future__ import annotations

import numpy as np


def _axes(dim, n1, n2, n3):
    return (n1, n2, n3) if dim == 3 else (n1, n3)


def neighbours(dim, n1, n2, n3):
    """[dim][2][N] neighbour index (side 0: -1 step, side 1: +1 step), -1 outside."""
    ax = _axes(dim, n1, n2, n3)
    N = int(np.prod(ax))
    idx = np.arange(N)
    stride = [1, ax[0], ax[0] * (ax[1] if dim == 3 else 1)][:dim]
    coord = []
    r = idx.copy()
    for d in range(dim):
        coord.append(r % ax[d])
        r = r // ax[d]
    nb = np.full((dim, 2, N), -1, dtype=np.int64)
    for d in range(dim):
        nb[d, 0] = np.where(coord[d] > 0, idx - stride[d], -1)
        nb[d, 1] = np.where(coord[d] < ax[d] - 1, idx + stride[d], -1)
    return nb


def segment_min(xi, si, x1, t1, x2, t2):
    """min over y on [x1, x2] of T(y) + si |xi - y| (T linear, t1 at x1, t2 at
    x2): the interior stationary point if it lies inside, else an end point.
    Vectorised over the leading axis; infinite end values give inf."""
    e = x2 - x1
    d0 = xi - x1
    a = np.sum(e * e, axis=-1)
    b = np.sum(d0 * e, axis=-1)
    c = np.sum(d0 * d0, axis=-1)
    best = np.minimum(t1 + si * np.sqrt(c), t2 + si * np.sqrt(np.sum((xi - x2) ** 2, axis=-1)))
    with np.errstate(invalid="ignore", divide="ignore"):
        delta = t2 - t1
        ok = np.isfinite(t1) & np.isfinite(t2) & (a * si * si > delta * delta)
        rperp2 = np.maximum(c - b * b / a, 0.0)
        rn = np.sqrt(rperp2) / np.sqrt(1.0 - delta * delta / (a * si * si))
        lam = b / a - (rn / si) * delta / a
        inside = ok & (lam > 0.0) & (lam < 1.0)
        val = t1 + lam * delta + si * rn
    return np.where(inside, np.minimum(best, val), best)


def triangle_min(xi, si, x1, t1, x2, t2, x3, t3):
    """min over y in the triangle (x1, x2, x3) of T(y) + si |xi - y|: the
    interior stationary point if inside, else the minimum over its edges."""
    best = np.minimum(np.minimum(segment_min(xi, si, x1, t1, x2, t2), segment_min(xi, si, x1, t1, x3, t3)),
                      segment_min(xi, si, x2, t2, x3, t3))
    e2, e3, d0 = x2 - x1, x3 - x1, xi - x1
    g22 = np.sum(e2 * e2, axis=-1)
    g23 = np.sum(e2 * e3, axis=-1)
    g33 = np.sum(e3 * e3, axis=-1)
    h2 = np.sum(e2 * d0, axis=-1)
    h3 = np.sum(e3 * d0, axis=-1)
    det = g22 * g33 - g23 * g23
    with np.errstate(invalid="ignore", divide="ignore"):
        # mu: barycentric coordinates (on e2, e3) of the projection of xi
        mu2 = (g33 * h2 - g23 * h3) / det
        mu3 = (g22 * h3 - g23 * h2) / det
        rperp2 = np.maximum(np.sum(d0 * d0, axis=-1) - (mu2 * h2 + mu3 * h3), 0.0)
        d2, d3 = t2 - t1, t3 - t1
        # q = delta^T Gm^{-1} delta
        i2 = (g33 * d2 - g23 * d3) / det
        i3 = (g22 * d3 - g23 * d2) / det
        q = d2 * i2 + d3 * i3
        ok = np.isfinite(t1) & np.isfinite(t2) & np.isfinite(t3) & (det > 0) & (si * si > q)
        rn = np.sqrt(rperp2) / np.sqrt(1.0 - q / (si * si))
        l2 = mu2 - (rn / si) * i2
        l3 = mu3 - (rn / si) * i3
        inside = ok & (l2 > 0.0) & (l3 > 0.0) & (l2 + l3 < 1.0)
        val = t1 + l2 * d2 + l3 * d3 + si * rn
    return np.where(inside, np.minimum(best, val), best)


def update(dim, nb, X, s, T):
    """The semi-Lagrangian update F(T) at every node (seeds not excluded)."""
    N = X.shape[0]
    big = np.inf
    best = np.full(N, big)
    nbr_x = []
    for d in range(dim):
        for side in range(2):
            k = nb[d, side]
            has = k >= 0
            kk = np.where(has, k, 0)
            xk = X[kk]
            tk = np.where(has, T[kk], big)
            nbr_x.append((d, side, xk, tk))
            best = np.minimum(best, np.where(has, tk + s * np.sqrt(np.sum((X - xk) ** 2, axis=1)), big))
    by_axis = {}
    for d, side, xk, tk in nbr_x:
        by_axis.setdefault(d, []).append((xk, tk))
    sc = s
    for a in range(dim):
        for b in range(a + 1, dim):
            for xa, ta in by_axis[a]:
                for xb, tb in by_axis[b]:
                    best = np.minimum(best, segment_min(X, sc, xa, ta, xb, tb))
    if dim == 3:
        for x0, t0 in by_axis[0]:
            for x1, t1 in by_axis[1]:
                for x2, t2 in by_axis[2]:
                    best = np.minimum(best, triangle_min(X, sc, x0, t0, x1, t1, x2, t2))
    return best


def seeds(dim, n1, n2, n3, X, s, src, radius):
    """(seed nodes, their straight-ray times) around the source node."""
    ax = _axes(dim, n1, n2, n3)
    N = int(np.prod(ax))
    idx = np.arange(N)
    coord, r = [], idx.copy()
    for d in range(dim):
        coord.append(r % ax[d])
        r = r // ax[d]
    m = np.ones(N, bool)
    for d in range(dim):
        m &= np.abs(coord[d] - coord[d][src]) <= radius
    nodes = np.nonzero(m)[0]
    t = 0.5 * (s[src] + s[nodes]) * np.sqrt(np.sum((X[nodes] - X[src]) ** 2, axis=1))
    t[nodes == src] = 0.0
    return nodes, t


def solve(dim, n1, n2, n3, X, s, src, radius=2, order="jacobi", max_iter=100000):
    """Iterate the update from T = +inf off the seeds until nothing changes.
    order: "jacobi" (all nodes from the previous iterate) or "gauss-seidel"
    (natural node order, in place, alternating with the reverse order).
    Returns (T, iterations)."""
    N = n1 * n2 * n3
    X = np.asarray(X, dtype=np.float64).reshape(N, dim)
    s = np.asarray(s, dtype=np.float64)
    sn, st = seeds(dim, n1, n2, n3, X, s, src, radius)
    return solve_seeded(dim, n1, n2, n3, X, s, sn, st, order, max_iter)


def solve_point(dim, n1, n2, n3, X, s, xi, rho, order="jacobi", max_iter=100000):
    """The same for a source at logical coordinates xi with a seed region of
    max-norm radius rho (the seeds of oracle.source: straight-ray times with
    s_src, x_src multilinear over xi's cell)."""
    from .source import seed_traveltime
    N = n1 * n2 * n3
    X = np.asarray(X, dtype=np.float64).reshape(N, dim)
    s = np.asarray(s, dtype=np.float64)
    sn, st, _, _ = seed_traveltime(dim, n1, n2, n3, X, s, np.asarray(xi, dtype=np.float64), rho)
    return solve_seeded(dim, n1, n2, n3, X, s, sn, st, order, max_iter)


def solve_seeded(dim, n1, n2, n3, X, s, sn, st, order="jacobi", max_iter=100000):
    """Iterate from T = st on the seed nodes sn and +inf elsewhere."""
    N = n1 * n2 * n3
    nb = neighbours(dim, n1, n2, n3)
    T = np.full(N, np.inf)
    T[sn] = st
    free = np.ones(N, bool)
    free[sn] = False
    for it in range(1, max_iter + 1):
        if order == "jacobi":
            new = np.where(free, np.minimum(T, update(dim, nb, X, s, T)), T)
            if np.array_equal(new, T):
                return T, it
            T = new
        else:
            changed = False
            seq = range(N) if it % 2 else range(N - 1, -1, -1)
            for i in seq:
                if not free[i]:
                    continue
                v = min(T[i], _update_one(dim, nb, X, s, T, i))
                if v != T[i]:
                    T[i] = v
                    changed = True
            if not changed:
                return T, it
    raise RuntimeError("no fixed point within max_iter")


def _update_one(dim, nb, X, s, T, i):
    """The update at node i alone (the same simplex minima)."""
    nbi = nb[:, :, i:i + 1]
    Xi = X[i:i + 1]
    best = np.inf
    for d in range(dim):
        for side in range(2):
            k = int(nbi[d, side, 0])
            if k >= 0:
                best = min(best, T[k] + s[i] * float(np.sqrt(np.sum((Xi[0] - X[k]) ** 2))))
    pts = {d: [(X[k][None], np.array([T[k]])) for k in nbi[d, :, 0] if k >= 0] for d in range(dim)}
    si = np.array([s[i]])
    for a in range(dim):
        for b in range(a + 1, dim):
            for xa, ta in pts[a]:
                for xb, tb in pts[b]:
                    best = min(best, float(segment_min(Xi, si, xa, ta, xb, tb)[0]))
    if dim == 3:
        for x0, t0 in pts[0]:
            for x1, t1 in pts[1]:
                for x2, t2 in pts[2]:
                    best = min(best, float(triangle_min(Xi, si, x0, t0, x1, t1, x2, t2)[0]))
    return best
