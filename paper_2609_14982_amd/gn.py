"""Regularised matrix-free Gauss-Newton tomography around the frozen transport
(Section 4.5 and Algorithm 1): the model is one velocity per cell, the data
are first-arrival times at the receivers of every source.

Outer iteration k (Algorithm 1):
  Phase I    nonlinear solve T_alpha(v_k) (a caller-supplied first-arrival
             solver s -> T[S][N]) and the frozen states of every source;
  Phase II   residual r_k = F(v_k) - d_obs (eq. (residual));
  Phase III  LSMR on the augmented system of eq. (augmented-ls),
                 K = [W_d J_k; lambda R; lambda S_k],  S_k = gamma diag(1/v_k),
             with J_k = P A^-1 C M applied on the GPU (M: ModelMap, the rest:
             Batch.apply_J / apply_JT) and K^T of eq. (augmented-actions);
  Phase IV   Armijo backtracking on the nonlinear weighted misfit
             0.5 ||W_d (F(v) - d_obs)||^2, then v_{k+1} = v_k + t_k dv_k.

R is the first difference between face-adjacent cells along every logical
axis (the model-increment roughness operator).  LSMR follows the recurrences
of Fong and Saunders (2011) with zero damping (the regularisation is in the
augmented operator).  Every transport application runs in the library's
kernels; the LSMR vector updates, R and the diagonal scalings are device
tensor operations on the batch stream.
"""
from __future__ import annotations


import numpy as np
import torch

from .binding import (FM_DS_BROADCAST, FM_FP64, FM_JT_SUMMED, FM_OUT_RECEIVERS, FM_W_RECEIVERS, Batch,
                      ModelMap, build_frozen_states)


class CellTomography:
    """Grid, acquisition and nonlinear solver of a cell-velocity tomography."""

    def __init__(self, dim, n1, n2, n3, G, src, rcv, solver, rcv_weights=None, nthreads=None):
        self.dim, self.n1, self.n2, self.n3 = dim, n1, n2, n3
        self.G = np.ascontiguousarray(G, dtype=np.float64)
        self.src = np.asarray(src, dtype=np.int64)
        self.rcv = np.asarray(rcv, dtype=np.int64)
        self.rcv_w = None if rcv_weights is None else np.asarray(rcv_weights, dtype=np.float64)
        self.solver = solver
        self.nthreads = nthreads
        self.S = int(self.src.shape[0])
        self.R = int(self.rcv.shape[0])
        ax = (n1, n2, n3) if dim == 3 else (n1, n3, 1)
        self.cells = tuple(max(a - 1, 1) for a in ax)     # cells per axis, axis 0 fastest

    @property
    def n_cells(self):
        return int(np.prod(self.cells))

    def sample(self, T):
        """P T for every source: [S][R]."""
        if self.rcv_w is None:
            return T[:, self.rcv]
        return np.einsum("srk,rk->sr", T[:, self.rcv], self.rcv_w)

    def forward(self, v):
        """F(v): (receiver times [S][R], T [S][N], nodal slowness [N], model map)."""
        m = ModelMap(self.dim, self.n1, self.n2, self.n3, v)
        s = m.slowness()
        T = np.ascontiguousarray(self.solver(s), dtype=np.float64)
        return self.sample(T), T, s, m

    def linearize(self, v, T, s, stream=None):
        states = build_frozen_states(self.dim, self.n1, self.n2, self.n3, self.G, T, s, self.src, self.rcv,
                                     nthreads=self.nthreads, rcv_weights=self.rcv_w)
        return Batch(states, 1, FM_FP64, stream=stream)


def roughness(p, cells):
    """R p: first differences of a cell field [Nc] along each cell axis, concatenated."""
    c0, c1, c2 = cells
    g = p.reshape(c2, c1, c0)
    parts = []
    if c0 > 1:
        parts.append((g[:, :, 1:] - g[:, :, :-1]).reshape(-1))
    if c1 > 1:
        parts.append((g[:, 1:, :] - g[:, :-1, :]).reshape(-1))
    if c2 > 1:
        parts.append((g[1:] - g[:-1]).reshape(-1))
    return torch.cat(parts)


def roughness_T(z, cells):
    """R^T z for z laid out as roughness() returns it."""
    c0, c1, c2 = cells
    out = torch.zeros((c2, c1, c0), dtype=z.dtype, device=z.device)
    o = 0
    if c0 > 1:
        n = c2 * c1 * (c0 - 1)
        d = z[o:o + n].reshape(c2, c1, c0 - 1)
        out[:, :, 1:] += d
        out[:, :, :-1] -= d
        o += n
    if c1 > 1:
        n = c2 * (c1 - 1) * c0
        d = z[o:o + n].reshape(c2, c1 - 1, c0)
        out[:, 1:, :] += d
        out[:, :-1, :] -= d
        o += n
    if c2 > 1:
        n = (c2 - 1) * c1 * c0
        d = z[o:o + n].reshape(c2 - 1, c1, c0)
        out[1:] += d
        out[:-1] -= d
    return out.reshape(-1)


class AugmentedOperator:
    """K = [W_d J; lambda R; lambda S] and K^T (eq. (augmented-actions)) at one
    frozen state; vectors are device tensors (model [Nc], data [S*R + nR + Nc])."""

    def __init__(self, prob: CellTomography, batch: Batch, mmap: ModelMap, wd, v, lam, gamma):
        dev = torch.device("cuda")
        self.prob, self.batch, self.mmap = prob, batch, mmap
        self.wd = torch.as_tensor(wd, dtype=torch.float64, device=dev).reshape(-1)
        self.sdiag = gamma / torch.as_tensor(v, dtype=torch.float64, device=dev)
        self.lam = float(lam)
        self.n_data = prob.S * prob.R
        self.n_rough = int(roughness(torch.zeros(prob.n_cells, dtype=torch.float64, device=dev),
                                     prob.cells).numel())
        N = batch.N
        self._ds = torch.empty((N, 1), dtype=torch.float64, device=dev)
        self._d = torch.empty((prob.S, prob.R, 1), dtype=torch.float64, device=dev)
        self._g = torch.empty((N, 1), dtype=torch.float64, device=dev)
        self._gc = torch.empty((prob.n_cells, 1), dtype=torch.float64, device=dev)

    @property
    def shape(self):
        return (self.n_data + self.n_rough + self.prob.n_cells, self.prob.n_cells)

    def J(self, p):
        self.mmap.apply(p.reshape(-1, 1).contiguous(), self._ds)
        self.batch.apply_J(self._ds, FM_DS_BROADCAST, self._d, FM_OUT_RECEIVERS)
        return self._d.reshape(-1)

    def JT(self, y):
        self.batch.apply_JT(y.reshape(self.prob.S, self.prob.R, 1).contiguous(), FM_W_RECEIVERS, self._g,
                            FM_JT_SUMMED)
        self.mmap.apply_T(self._g, self._gc)
        return self._gc.reshape(-1)

    def matvec(self, p):
        return torch.cat([self.wd * self.J(p), self.lam * roughness(p, self.prob.cells), self.lam * self.sdiag * p])

    def rmatvec(self, y):
        a, b = self.n_data, self.n_data + self.n_rough
        return (self.JT(self.wd * y[:a]) + self.lam * roughness_T(y[a:b], self.prob.cells)
                + self.lam * self.sdiag * y[b:])


def lsmr(op, b, n_iter, atol=0.0, btol=0.0, check_every=8):
    """LSMR for min ||op x - b|| from x = 0 (the recurrences of Fong and
    Saunders, 2011, with zero damping - the regularisation is inside the
    augmented operator), at most n_iter iterations.

    Stopping (their tests, with the norm estimates of the same recurrences):
    ||op^T r|| <= atol ||op|| ||r||  (a least-squares solution to the Krylov
    optimality tolerance atol; Section 5.3 uses 1e-4), or
    ||r|| <= btol ||b|| + atol ||op|| ||x||  (a compatible system).  Every
    scalar stays on the device: a converged column freezes x on the device,
    and the host reads the stop flag only every check_every iterations, so
    the loop has no per-iteration synchronisation.
    Returns (x, ||b - op x||, iterations used, info dict)."""
    dev, dt = b.device, b.dtype
    zero = torch.zeros((), dtype=dt, device=dev)
    one = torch.ones((), dtype=dt, device=dev)

    def safe_div(a, c):
        return torch.where(c != 0, a / torch.where(c != 0, c, one), zero)

    beta = torch.linalg.vector_norm(b)
    normb = beta
    x = torch.zeros(op.shape[1], dtype=dt, device=dev)
    u = safe_div(one, beta) * b
    v = op.rmatvec(u)
    alpha = torch.linalg.vector_norm(v)
    v = safe_div(one, alpha) * v
    # bidiagonalisation and the two rotations
    zetabar = alpha * beta
    alphabar = alpha
    rho, rhobar, cbar, sbar = one.clone(), one.clone(), one.clone(), zero.clone()
    h = v.clone()
    hbar = torch.zeros_like(v)
    # estimates of ||r|| (betadd, betad, rhodold, tautildeold, thetatilde, zeta)
    betadd, betad, rhodold = beta.clone(), zero.clone(), one.clone()
    tautildeold, thetatilde, zeta = zero.clone(), zero.clone(), zero.clone()
    normA2 = alpha * alpha
    # an exact zero residual (beta = 0) or gradient (alpha = 0) at the start
    active = (beta > 0) & (alpha > 0)
    itn = torch.zeros((), dtype=torch.int64, device=dev)
    normr = beta.clone()
    normAr = alpha * beta
    for k in range(n_iter):
        if k % check_every == 0 and not bool(active):
            break
        # beta u = op v - alpha u ; alpha v = op^T u - beta v
        u = op.matvec(v) - alpha * u
        beta = torch.linalg.vector_norm(u)
        u = safe_div(one, beta) * u
        v = op.rmatvec(u) - beta * v
        alpha = torch.linalg.vector_norm(v)
        v = safe_div(one, alpha) * v
        # rotation P_k
        rhoold = rho
        rho = torch.sqrt(alphabar * alphabar + beta * beta)
        c, s = safe_div(alphabar, rho), safe_div(beta, rho)
        thetanew = s * alpha
        alphabar = c * alpha
        # rotation Pbar_k
        rhobarold = rhobar
        zetaold = zeta
        thetabar = sbar * rho
        rhotemp = cbar * rho
        rhobar = torch.sqrt(rhotemp * rhotemp + thetanew * thetanew)
        cbar, sbar = safe_div(rhotemp, rhobar), safe_div(thetanew, rhobar)
        zeta = cbar * zetabar
        zetabar = -sbar * zetabar
        # h, hbar, x (x only while the column is active)
        hbar = h - safe_div(thetabar * rho, rhoold * rhobarold) * hbar
        x = torch.where(active, x + safe_div(zeta, rho * rhobar) * hbar, x)
        h = v - safe_div(thetanew, rho) * h
        # ||r|| estimate (zero damping: the damping rotation is the identity)
        betahat = c * betadd
        betadd = -s * betadd
        thetatildeold = thetatilde
        rhotildeold = torch.sqrt(rhodold * rhodold + thetabar * thetabar)
        ctildeold, stildeold = safe_div(rhodold, rhotildeold), safe_div(thetabar, rhotildeold)
        thetatilde = stildeold * rhobar
        rhodold = ctildeold * rhobar
        betad = -stildeold * betad + ctildeold * betahat
        tautildeold = safe_div(zetaold - thetatildeold * tautildeold, rhotildeold)
        taud = safe_div(zeta - thetatilde * tautildeold, rhodold)
        nr = torch.sqrt((betad - taud) ** 2 + betadd * betadd)
        # ||A|| estimate, ||A^T r||, ||x||
        normA2 = normA2 + beta * beta
        normA = torch.sqrt(normA2)
        normA2 = normA2 + alpha * alpha
        nAr = torch.abs(zetabar)
        normx = torch.linalg.vector_norm(x)
        normr = torch.where(active, nr, normr)
        normAr = torch.where(active, nAr, normAr)
        itn = itn + active.to(torch.int64)
        test1 = safe_div(nr, normb)
        den = normA * nr
        test2 = torch.where(den != 0, nAr / torch.where(den != 0, den, one), torch.full_like(den, float("inf")))
        t1 = test1 / (1 + safe_div(normA * normx, normb))
        rtol = btol + atol * safe_div(normA * normx, normb)
        # the two tests, and their machine-precision limits
        done = (test2 <= atol) | (test1 <= rtol) | (1 + test2 <= 1) | (1 + t1 <= 1)
        active = active & ~done
    info = {"iterations": int(itn), "normr_est": float(normr), "normAr_est": float(normAr),
            "converged": not bool(active)}
    return x, float(torch.linalg.vector_norm(b - op.matvec(x))), info["iterations"], info


def wrms(wd, r):
    """Weighted RMS data residual sqrt(mean((W_d r)^2)) (Section 5.4)."""
    return float(np.sqrt(np.mean((np.asarray(wd) * np.asarray(r)) ** 2)))


def data_weights(d_obs, sigma_abs, sigma_rel):
    """W_d: inverse standard deviation of each datum, an absolute floor and a
    relative term in quadrature."""
    return 1.0 / np.sqrt(sigma_abs ** 2 + (sigma_rel * d_obs) ** 2)


def gauss_newton(prob: CellTomography, v0, d_obs, lam, gamma, sigma_abs, sigma_rel, k_max=10, n_lsmr=100,
                 lsmr_atol=1e-4, lsmr_btol=1e-4, outer_rtol=0.01, c1=1e-4, max_halvings=8):
    """Algorithm 1: at most k_max + 1 outer iterations.  Phase II stops when
    the relative reduction of the weighted RMS residual between successive
    outer iterations falls below outer_rtol (Section 5.4 uses 1 %); LSMR stops
    at the Krylov optimality tolerance lsmr_atol (Section 5.3: 1e-4) or after
    n_lsmr iterations; Armijo halves the step from t = 1 while the nonlinear
    weighted misfit does not fall by c1 t |slope|.  Returns (v, history): one
    record per outer iteration (weighted misfit and WRMS at v_k, step length,
    LSMR iterations and residual, the stop reason on the last)."""
    wd = data_weights(np.asarray(d_obs, dtype=np.float64), sigma_abs, sigma_rel)
    v = np.ascontiguousarray(v0, dtype=np.float64)
    hist = []
    dev = torch.device("cuda")
    pred, T, s, mmap = prob.forward(v)
    prev_wrms = None
    for k in range(k_max + 1):
        # Phase II: residual and the outer stopping test
        r = pred - d_obs
        phi = 0.5 * float(np.sum((wd * r) ** 2))
        w = wrms(wd, r)
        rec = {"k": k, "misfit": phi, "wrms": w}
        hist.append(rec)
        if prev_wrms is not None and (prev_wrms - w) < outer_rtol * prev_wrms:
            rec["stop"] = "relative WRMS reduction below %g" % outer_rtol
            break
        if k == k_max:
            rec["stop"] = "k_max"
            break
        prev_wrms = w
        # Phase I (at v_k) and III: frozen states, LSMR on the augmented system
        batch = prob.linearize(v, T, s)
        K = AugmentedOperator(prob, batch, mmap, wd, v, lam, gamma)
        rhs = torch.zeros(K.shape[0], dtype=torch.float64, device=dev)
        rhs[:K.n_data] = torch.from_numpy(-(wd * r).reshape(-1)).to(dev)
        dv, res, its, info = lsmr(K, rhs, n_lsmr, atol=lsmr_atol, btol=lsmr_btol)
        # directional derivative of the weighted misfit: (J^T W_d^2 r) . dv
        gradv = K.JT(torch.from_numpy((wd * wd * r).reshape(-1)).to(dev))
        slope = float(torch.dot(gradv, dv))
        batch.status()
        dv = dv.cpu().numpy()
        batch.free()
        rec.update({"lsmr_iterations": its, "lsmr_converged": info["converged"], "lsmr_residual": res,
                    "lsmr_rhs": float(torch.linalg.vector_norm(rhs)), "slope": slope})
        # Phase IV: Armijo on the nonlinear weighted misfit
        t, accepted = 1.0, None
        for _h in range(max_halvings + 1):
            vt = v + t * dv
            if np.all(vt > 0):
                pt, Tt, st, mt = prob.forward(vt)
                phit = 0.5 * float(np.sum((wd * (pt - d_obs)) ** 2))
                if phit <= phi + c1 * t * slope:
                    accepted = (vt, pt, Tt, st, mt)
                    break
                mt.free()
            t *= 0.5
        rec["step"] = t if accepted else 0.0
        if accepted is None:
            rec["stop"] = "no step satisfies the Armijo condition"
            break
        mmap.free()
        v, pred, T, s, mmap = accepted
    mmap.free()
    return v, hist
