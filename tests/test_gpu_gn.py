"""The Gauss-Newton driver of Section 4.5 / Algorithm 1 on the GPU: cell
velocities, the frozen transport, LSMR on the augmented operator, Armijo.

* LSMR (the driver's, on K = [W_d J M; lambda R; lambda S_k] applied through
  the library) against scipy's LSMR on the oracle's explicit operator (oracle
  J, explicit sparse M and R, diagonal S): the same 12 iterations give the
  same model increment to 1e-9;
* two outer iterations on a 2-D grid with a seeded velocity anomaly: the
  first increment is a descent direction with an accepted step, every
  accepted step satisfies the Armijo condition, and the weighted misfit
  falls by more than half;
* Algorithm 1 to its own stop: LSMR at the Krylov optimality tolerance
  1e-4 (Section 5.3) and the outer loop ending when the relative WRMS
  reduction falls below 1 % (Section 5.4) - every earlier outer iteration
  reduced it by at least 1 %.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from helpers import oracle_ops
from oracle.model_map import model_map_matrix
from test_gn_cpu import _explicit_R

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")
gn = pytest.importorskip("paper_2609_14982_amd.gn")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem():
    wl = W.grids.deformed_2d(61, 31, 6100, 0.3, 2, S=3, B=1, R=12, name="gn 61x31")
    v0 = W.cell_velocities(wl)
    m = fm.ModelMap(2, wl.n1, 1, wl.n3, v0)
    wl.s = m.slowness()
    m.free()
    W.eikonal(wl)
    prob = gn.CellTomography(2, wl.n1, 1, wl.n3, wl.G, wl.src, wl.rcv, W.traveltime_solver(wl), nthreads=8)
    return wl, v0, prob


def test_lsmr_matches_scipy_on_oracle_operator(problem):
    wl, v0, prob = problem
    lam, gamma = 0.7, 0.5
    pred, T, s, mmap = prob.forward(v0)
    d_obs = pred + 1e-3 * np.random.default_rng(6101).standard_normal(pred.shape)
    wd = gn.data_weights(d_obs, 3e-4, 3e-3)
    batch = prob.linearize(v0, T, s)
    K = gn.AugmentedOperator(prob, batch, mmap, wd, v0, lam, gamma)
    b = np.zeros(K.shape[0])
    b[:K.n_data] = -(wd * (pred - d_obs)).reshape(-1)
    x, res, its, info = gn.lsmr(K, torch.from_numpy(b).to("cuda"), 12)
    assert its == 12
    x = x.cpu().numpy()

    ops = oracle_ops(wl)
    Mo = model_map_matrix(2, wl.n1, 1, wl.n3, v0)
    Ro = _explicit_R(prob.cells)
    Sd = gamma / v0
    wdf = wd.reshape(-1)

    def mv(p):
        ds = Mo @ p
        j = np.concatenate([O.apply_J(op, ds, "receivers") for op in ops])
        return np.concatenate([wdf * j, lam * (Ro @ p), lam * Sd * p])

    def rmv(y):
        a, c = K.n_data, K.n_data + Ro.shape[0]
        yd = (wdf * y[:a]).reshape(prob.S, prob.R)
        g = O.apply_JT_summed(ops, list(yd), "receivers")
        return Mo.T @ g + lam * (Ro.T @ y[a:c]) + lam * Sd * y[c:]

    A = spla.LinearOperator(K.shape, matvec=mv, rmatvec=rmv, dtype=np.float64)
    xr = spla.lsmr(A, b, damp=0.0, atol=0.0, btol=0.0, conlim=1e300, maxiter=12)[0]
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert abs(res - np.linalg.norm(b - mv(x))) <= 1e-9 * np.linalg.norm(b)
    batch.free()
    mmap.free()


def test_gauss_newton_descends(problem):
    wl, v0, prob = problem
    c0, c1, _ = prob.cells
    ci, ck = np.meshgrid(np.arange(c0), np.arange(c1), indexing="xy")
    bump = np.exp(-((ci - 0.5 * c0) ** 2 + (ck - 0.5 * c1) ** 2) / (2.0 * 6.0 ** 2)).reshape(-1)
    v_true = v0 * (1.0 + 0.06 * bump)
    d_obs = prob.forward(v_true)[0]
    v, hist = gn.gauss_newton(prob, v0, d_obs, lam=2.0, gamma=1.0, sigma_abs=3e-4, sigma_rel=3e-3,
                              k_max=2, n_lsmr=25, lsmr_atol=0.0, lsmr_btol=0.0, outer_rtol=0.0)
    print("misfits", [h["misfit"] for h in hist], "steps", [h.get("step") for h in hist], flush=True)
    # the first increment is a descent direction and its step is accepted;
    # later ones may find no step (the tangent is that of the continuous
    # equation, not of the fast-marching solver), and the driver then keeps
    # the last accepted model
    assert hist[0]["slope"] < 0.0 and hist[0]["step"] > 0.0 and hist[0]["lsmr_iterations"] == 25
    for a, b in zip(hist[:-1], hist[1:]):
        if a.get("step", 0.0) > 0.0:
            assert b["misfit"] <= a["misfit"] + 1e-4 * a["step"] * a["slope"]
    assert hist[-1]["misfit"] < 0.5 * hist[0]["misfit"]
    assert np.all(v > 0)


def test_gauss_newton_stops_on_wrms_reduction(problem):
    wl, v0, prob = problem
    c0, c1, _ = prob.cells
    ci, ck = np.meshgrid(np.arange(c0), np.arange(c1), indexing="xy")
    bump = np.exp(-((ci - 0.35 * c0) ** 2 + (ck - 0.5 * c1) ** 2) / (2.0 * 5.0 ** 2)).reshape(-1)
    v_true = v0 * (1.0 - 0.05 * bump)
    d_obs = prob.forward(v_true)[0]
    d_obs = d_obs + 3e-4 * np.random.default_rng(6102).standard_normal(d_obs.shape)
    v, hist = gn.gauss_newton(prob, v0, d_obs, lam=1.0, gamma=0.5, sigma_abs=3e-4, sigma_rel=3e-3,
                              k_max=12, n_lsmr=200, lsmr_atol=1e-4, lsmr_btol=1e-4, outer_rtol=0.01)
    ws = [h["wrms"] for h in hist]
    print("wrms", ws, "lsmr iterations", [h.get("lsmr_iterations") for h in hist], "stop", hist[-1]["stop"],
          flush=True)
    for h in hist[:-1]:
        assert h["lsmr_converged"] and h["lsmr_iterations"] < 200
    stop = hist[-1]["stop"]
    assert stop.startswith("relative WRMS") or stop.startswith("no step"), stop
    if stop.startswith("relative WRMS"):
        assert ws[-2] - ws[-1] < 0.01 * ws[-2]
    for k in range(1, len(ws) - 1):
        assert ws[k - 1] - ws[k] >= 0.01 * ws[k - 1]
    assert ws[-1] < ws[0]
