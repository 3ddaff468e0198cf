"""Differentiation wrapper and Gauss-Newton step over the frozen transport.

ReceiverTraveltime is a torch.autograd.Function for the map
    s (nodal slowness [N])  ->  receiver traveltimes [S][R]
whose forward pass runs a caller-supplied nonlinear first-arrival solver
(s -> T[S][N], the state of Section 2.1; GpuTraveltimeSolver runs the
library's GPU solver) and builds the frozen states
(Algorithm 1, Phase I), and whose backward pass applies the source-summed
transpose J^T = sum_alpha C_alpha A_alpha^{-T} P_alpha^T (Section 4.4) on the
GPU.  The tangent is the frozen face-upwind transport with the calibrated
right-hand side (Section 3.2); it is the derivative of the continuous state
equation, not of the particular nonlinear solver, so finite differences of
the solver agree with it to discretisation accuracy (exactly along the
uniform scaling direction ds = s, where both give T).

gauss_newton_step computes the Gauss-Newton increment of the data misfit
0.5 ||P T(s) - d||^2 by CGLS on J (Algorithm 1, with CGLS in
place of LSMR and no regularisation); the CGLS iterations run in the
library's kernels, captured as one HIP graph.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import (FM_DS_BROADCAST, FM_FP64, FM_JT_SUMMED, FM_OUT_RECEIVERS, FM_W_RECEIVERS, Batch, Cgls,
                      Eikonal, build_frozen_states)


class GpuTraveltimeSolver:
    """The nonlinear state on the GPU (fm_eikonal_*): a callable s [N] (host)
    -> T [S][N] (host) for sources on the given nodes, with seed regions of
    max-norm radius seed_radius (Algorithm 1, Phase I; Section 2.1)."""

    def __init__(self, dim, n1, n2, n3, X, src, seed_radius=2.0):
        self.dim, self.N = dim, n1 * n2 * n3
        axes = (n1, n2, n3) if dim == 3 else (n1, n3)
        src = np.asarray(src, dtype=np.int64)
        # logical coordinates of the source nodes (axis 0 fastest)
        xi = np.empty((src.size, dim))
        r = src.copy()
        for d in range(dim):
            xi[:, d] = r % axes[d]
            r = r // axes[d]
        self.xi = xi
        self.seed_radius = float(seed_radius)
        self.iterations = 0
        self._solver = Eikonal(dim, n1, n2, n3, X, src.size)

    def __call__(self, s: np.ndarray) -> np.ndarray:
        dev = torch.device("cuda")
        T = torch.empty((self.xi.shape[0], self.N), dtype=torch.float64, device=dev)
        self.iterations = self._solver.solve(torch.from_numpy(np.ascontiguousarray(s, dtype=np.float64)).to(dev),
                                             self.xi, self.seed_radius, T)
        return T.cpu().numpy()


class TransportProblem:
    """Grid, metric, sources, receivers and the nonlinear solver s -> T[S][N]."""

    def __init__(self, dim, n1, n2, n3, G, src, rcv, solver, nthreads=None):
        self.dim, self.n1, self.n2, self.n3 = dim, n1, n2, n3
        self.G = np.ascontiguousarray(G, dtype=np.float64)
        self.src = np.asarray(src, dtype=np.int64)
        self.rcv = np.asarray(rcv, dtype=np.int64)
        self.solver = solver
        self.nthreads = nthreads
        self.N = n1 * n2 * n3
        self.S = int(self.src.shape[0])
        self.R = int(self.rcv.shape[0])

    def linearize(self, s: np.ndarray, B: int = 1, stream=None):
        """Nonlinear solve at s and Phase I setup: returns (T [S][N], batch)."""
        s = np.ascontiguousarray(s, dtype=np.float64)
        T = np.ascontiguousarray(self.solver(s), dtype=np.float64)
        self.last_T = T     # the state of the latest linearisation (for checks against an oracle)
        states = build_frozen_states(self.dim, self.n1, self.n2, self.n3, self.G, T, s, self.src,
                                     self.rcv, nthreads=self.nthreads)
        return T, Batch(states, B, FM_FP64, stream=stream)


class ReceiverTraveltime(torch.autograd.Function):
    """s [N] -> P T(s) [S][R]; backward = J^T (source-summed) on the GPU."""

    @staticmethod
    def forward(ctx, s, problem: TransportProblem):
        T, batch = problem.linearize(s.detach().double().cpu().numpy())
        ctx.batch = batch
        ctx.problem = problem
        ctx.s_device = s.device
        ctx.s_dtype = s.dtype
        return torch.from_numpy(np.ascontiguousarray(T[:, problem.rcv])).to(device=s.device, dtype=s.dtype)

    @staticmethod
    def backward(ctx, grad):
        problem, batch = ctx.problem, ctx.batch
        dev = torch.device("cuda")
        g = grad.detach().to(device=dev, dtype=torch.float64).reshape(problem.S, problem.R, 1).contiguous()
        out = torch.empty((problem.N, 1), device=dev, dtype=torch.float64)
        batch.apply_JT(g, FM_W_RECEIVERS, out, FM_JT_SUMMED)
        batch.status()      # synchronises; raises if a level wait of the launch gave up
        return out.reshape(problem.N).to(device=ctx.s_device, dtype=ctx.s_dtype), None


def receiver_traveltime(s: torch.Tensor, problem: TransportProblem) -> torch.Tensor:
    return ReceiverTraveltime.apply(s, problem)


def apply_J_receivers(batch: Batch, p: torch.Tensor) -> torch.Tensor:
    """J p for a model block p [N][B] -> [S][R][B]."""
    out = torch.empty((batch.S, batch.R, batch.B), device=p.device, dtype=p.dtype)
    batch.apply_J(p.contiguous(), FM_DS_BROADCAST, out, FM_OUT_RECEIVERS)
    return out


def apply_JT_summed(batch: Batch, y: torch.Tensor) -> torch.Tensor:
    """J^T y for receiver data y [S][R][B] -> [N][B]."""
    out = torch.empty((batch.N, batch.B), device=y.device, dtype=y.dtype)
    batch.apply_JT(y.contiguous(), FM_W_RECEIVERS, out, FM_JT_SUMMED)
    return out


def cgls(batch: Batch, r: torch.Tensor, n_iter: int, graph: bool = True):
    """CGLS for min ||J x - r|| per column: r [S][R][B] -> (x [N][B], residual
    norms [n_iter + 1][B]).  Every step runs in the library (fm_cgls): with
    graph=True the n_iter iterations are captured once as a HIP graph and
    replayed, so the loop has no host round trip."""
    solver = Cgls(batch, max_iter=n_iter)
    home = batch._stream
    # a graph is captured from a stream of its own (the null stream cannot be
    # captured); it starts after the caller's pending work on that stream
    side = torch.cuda.Stream() if graph and home.cuda_stream == 0 else None
    try:
        if side is not None:
            side.wait_stream(home)
            batch.set_stream(side)
        solver.start(r.contiguous())
        if n_iter > 0:
            if graph:
                solver.capture(n_iter)
                solver.replay()
            else:
                solver.iterate(n_iter)
        batch.status()
        x = solver.x()
        norms = torch.sqrt(solver.history()[:n_iter + 1])
    finally:
        if side is not None:
            home.wait_stream(side)
            batch.set_stream(home)
        solver.free()
    return x, norms


def gauss_newton_step(problem: TransportProblem, s: np.ndarray, d_obs: np.ndarray, n_iter: int = 30):
    """One matrix-free Gauss-Newton increment ds for 0.5 ||P T(s) - d_obs||^2:
    linearise at s, then CGLS on J ds = d_obs - P T(s).  Returns (ds, misfit
    before, CGLS residual norms)."""
    dev = torch.device("cuda")
    T, batch = problem.linearize(s)
    r = d_obs - T[:, problem.rcv]
    rt = torch.from_numpy(np.ascontiguousarray(r)[:, :, None]).to(dev)
    ds, norms = cgls(batch, rt, n_iter)
    torch.cuda.synchronize()
    out = ds[:, 0].cpu().numpy()
    batch.free()
    return out, 0.5 * float(np.sum(r * r)), norms[:, 0].cpu().numpy()
