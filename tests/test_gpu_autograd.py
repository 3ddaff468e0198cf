"""torch.autograd.Function for slowness -> receiver traveltime and the CGLS
Gauss-Newton step (the differentiation part of the benchmark statement).

* The backward pass equals the oracle's source-summed transpose applied to the
  output gradient (Section 4.4) to 1e-11.
* Central finite differences of the nonlinear solver (step 1e-6 relative):
  exact agreement with J along the uniform scaling direction ds = s (both
  give T, Section 3.2); along smooth directions agreement is at the
  discretisation level only (the tangent is the derivative of the continuous
  state equation, not of this solver), recorded here as <= 5 %.
* GPU CGLS iterates equal CGLS in NumPy on the oracle's operator, and a
  Gauss-Newton step reduces the data misfit of a perturbed model.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.assembly import assemble_workload

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")
from paper_2609_14982_amd import autograd as AG  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem():
    wl = W.small_3d(41, 41, 21, seed=77, S=4, B=1, with_T=True)
    prob = AG.TransportProblem(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.src, wl.rcv,
                               W.traveltime_solver(wl))
    return wl, prob


def test_backward_is_oracle_transpose(problem):
    wl, prob = problem
    print("case autograd backward 41x41x21, S=4", flush=True)
    s = torch.tensor(wl.s, dtype=torch.float64, requires_grad=True)
    d_obs = wl.T[:, wl.rcv] + 1e-3 * np.random.default_rng(3).standard_normal((wl.S, wl.rcv.shape[0]))
    pred = AG.receiver_traveltime(s, prob)
    loss = 0.5 * torch.sum((pred - torch.from_numpy(d_obs)) ** 2)
    loss.backward()
    grad = s.grad.numpy()
    resid = pred.detach().numpy() - d_obs
    ops = [assemble_workload(wl, a) for a in range(wl.S)]
    ref = O.apply_JT_summed(ops, list(resid), "receivers")
    assert np.linalg.norm(grad - ref) / np.linalg.norm(ref) <= 1e-11


def _fd(prob, s, ds, eps):
    Tp = prob.solver(s + eps * ds)
    Tm = prob.solver(s - eps * ds)
    return (Tp[:, prob.rcv] - Tm[:, prob.rcv]) / (2 * eps)


def test_finite_differences_of_the_solver(problem):
    wl, prob = problem
    T, batch = prob.linearize(wl.s)
    dev = torch.device("cuda")
    x, y, z = wl.X[:, 0], wl.X[:, 1], wl.X[:, 2]
    smooth = wl.s * 0.02 * np.sin(np.pi * x / 4) * np.cos(np.pi * y / 4) * (1 + z / 2)
    for ds, tol in ((wl.s.copy(), 1e-6), (smooth, 5e-2)):
        eps = 1e-6 * np.abs(wl.s).max() / np.abs(ds).max()
        fd = _fd(prob, wl.s, ds, eps)
        Jd = AG.apply_J_receivers(batch, torch.from_numpy(ds[:, None]).to(dev))[:, :, 0].cpu().numpy()
        err = np.linalg.norm(Jd - fd) / np.linalg.norm(fd)
        print(f"fd vs J: {err:.3e} (bar {tol:g})", flush=True)
        assert err <= tol
    batch.free()


def test_cgls_matches_numpy_on_oracle_operator(problem):
    wl, prob = problem
    T, batch = prob.linearize(wl.s)
    ops = [assemble_workload(wl, a) for a in range(wl.S)]
    rng = np.random.default_rng(9)
    r = rng.standard_normal((wl.S, wl.rcv.shape[0]))
    n_it = 6
    x_gpu, norms = AG.cgls(batch, torch.from_numpy(r[:, :, None]).to("cuda"), n_it)
    x_gpu = x_gpu[:, 0].cpu().numpy()

    def J(p):
        return np.stack([O.apply_J(op, p, "receivers") for op in ops])

    def JT(yy):
        return O.apply_JT_summed(ops, list(yy), "receivers")
    x = np.zeros(wl.N)
    res = r.copy()
    sv = JT(res)
    p = sv.copy()
    gamma = sv @ sv
    for _ in range(n_it):
        q = J(p)
        alpha = gamma / np.sum(q * q)
        x += alpha * p
        res -= alpha * q
        sv = JT(res)
        gnew = sv @ sv
        p = sv + (gnew / gamma) * p
        gamma = gnew
    assert np.linalg.norm(x_gpu - x) / np.linalg.norm(x) <= 1e-9
    assert np.all(np.diff(norms[:, 0].cpu().numpy()) <= 1e-12)
    batch.free()


def test_gauss_newton_step_reduces_misfit(problem):
    wl, prob = problem
    rng = np.random.default_rng(21)
    x, y, z = wl.X[:, 0], wl.X[:, 1], wl.X[:, 2]
    blob = 0.05 * np.exp(-((x - 2.0) ** 2 + (y - 2.0) ** 2 + (z - 1.0) ** 2) / (2 * 0.6 ** 2))
    s_true = wl.s * (1.0 + blob)
    d_obs = prob.solver(s_true)[:, prob.rcv]
    ds, misfit0, norms = AG.gauss_newton_step(prob, wl.s, d_obs, n_iter=30)
    T1 = prob.solver(wl.s + ds)
    misfit1 = 0.5 * float(np.sum((T1[:, prob.rcv] - d_obs) ** 2))
    print(f"GN step: misfit {misfit0:.3e} -> {misfit1:.3e}", flush=True)
    assert misfit1 < 0.5 * misfit0
    assert rng is not None
