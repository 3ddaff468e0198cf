"""The Gauss-Newton configuration at full size (c4's 201 x 201 x 101 grid,
64 sources x 400 receivers): a true model with six seeded +-5 % slowness
anomalies gives d_obs = P T(s_true) by the first-arrival solver; one
matrix-free Gauss-Newton step (CGLS, 30 iterations of J and the
source-summed J^T on the GPU, Algorithm 1) must reduce the
nonlinear data misfit, and the CGLS residual norms must not increase."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")
from paper_2609_14982_amd import autograd as AG  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_c5_gauss_newton_step_full_size():
    print("case c5: 201x201x101, S=64, R=400, CGLS 30", flush=True)
    wl = W.config("c4", with_T=False)
    prob = AG.TransportProblem(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.src, wl.rcv,
                               W.traveltime_solver(wl, nthreads=16), nthreads=16)
    s_true = W.perturbed_model(wl, 5000)
    d_obs = prob.solver(s_true)[:, prob.rcv]
    print("data computed", flush=True)
    ds, misfit0, norms = AG.gauss_newton_step(prob, wl.s, d_obs, n_iter=30)
    T1 = prob.solver(wl.s + ds)
    misfit1 = 0.5 * float(np.sum((T1[:, prob.rcv] - d_obs) ** 2))
    print(f"c5 GN step: misfit {misfit0:.4e} -> {misfit1:.4e}; CGLS residual {norms[0]:.3e} -> {norms[-1]:.3e}",
          flush=True)
    assert np.all(np.diff(norms) <= 1e-12 * norms[0])
    assert norms[-1] < 0.5 * norms[0]
    assert misfit1 < 0.5 * misfit0
