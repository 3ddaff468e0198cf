"""The LSQR harness (Krylov inner loop over the paired actions, Algorithm 1,
Section 4.5) on the GPU.

* Its iterates match scipy's LSQR run on the oracle's J and J^T (stacked
  sources, source-summed transpose) column by column.
* A captured HIP graph of n iterations, replayed with eager work and
  synchronisation between replays, reproduces the eager iterations bit for
  bit, on every replay.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from helpers import oracle_ops, states_for

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem():
    wl = W.grids.deformed_2d(61, 31, 91, 0.4, 2, S=3, B=4, R=12, name="lsqr-mini")
    W.eikonal(wl)
    return wl, states_for(fm, wl), oracle_ops(wl)


def _stacked_operator(wl, ops):
    S, R, N = wl.S, wl.rcv.shape[0], wl.N

    def mv(p):
        return np.concatenate([O.apply_J(op, p, "receivers") for op in ops])

    def rmv(y):
        y = y.reshape(S, R)
        return O.apply_JT_summed(ops, list(y), "receivers")

    return spla.LinearOperator((S * R, N), matvec=mv, rmatvec=rmv, dtype=np.float64)


def test_lsqr_matches_scipy_on_oracle_operator(problem):
    wl, states, ops = problem
    B, n_it = 4, 8
    rng = np.random.default_rng(5)
    d = rng.standard_normal((wl.S, wl.rcv.shape[0], B))
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = fm.Batch(states, B, fm.FM_FP64, stream=stream)
        L = fm.Lsqr(batch)
        L.start(torch.from_numpy(d).to(dev))
        L.iterate(n_it)
        x = L.x().cpu().numpy()
        phibar = np.abs(L.scalars().cpu().numpy()[3])
    A = _stacked_operator(wl, ops)
    for b in range(B):
        res = spla.lsqr(A, d[:, :, b].reshape(-1), damp=0.0, atol=0.0, btol=0.0, conlim=1e300,
                        iter_lim=n_it)
        xr, itn = res[0], res[2]
        assert itn == n_it
        assert np.linalg.norm(x[:, b] - xr) / np.linalg.norm(xr) <= 1e-9
        # |phibar| is the residual norm ||d - J x||
        r = d[:, :, b].reshape(-1) - A.matvec(x[:, b])
        assert abs(np.linalg.norm(r) - phibar[b]) <= 1e-9 * np.linalg.norm(d[:, :, b])
    L.free()
    batch.free()


def test_lsqr_graph_replays_match_eager(problem):
    wl, states, ops = problem
    B = 4
    rng = np.random.default_rng(6)
    d = torch.from_numpy(rng.standard_normal((wl.S, wl.rcv.shape[0], B))).to("cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = fm.Batch(states, B, fm.FM_FP64, stream=stream)
        L = fm.Lsqr(batch)
        # eager reference: start + 6 iterations
        L.start(d)
        L.iterate(6)
        x_ref = L.x().cpu().numpy()
        s_ref = L.scalars().cpu().numpy()
        # graph of 3 iterations, replayed twice per run, three runs
        L.start(d)
        L.capture(3)
        for run in range(3):
            L.start(d)
            torch.cuda.synchronize()
            L.replay()
            torch.cuda.synchronize()
            junk = torch.randn(1000, device="cuda").sum().item()      # eager work in between
            assert np.isfinite(junk)
            L.replay()
            torch.cuda.synchronize()
            assert np.array_equal(L.x().cpu().numpy(), x_ref), run
            assert np.array_equal(L.scalars().cpu().numpy(), s_ref), run
    L.free()
    batch.free()


def _cgls_numpy(mv, rmv, d, n_it):
    """CGLS written out on an explicit operator: x = 0, r = d, s = J^T r,
    p = s; q = J p, alpha = |s|^2 / |q|^2, x += alpha p, r -= alpha q,
    s = J^T r, p = s + (|s'|^2 / |s|^2) p."""
    x = np.zeros(rmv(d).shape[0])
    r = d.copy()
    s = rmv(r)
    p = s.copy()
    gamma = s @ s
    norms = [np.linalg.norm(r)]
    for _ in range(n_it):
        q = mv(p)
        alpha = gamma / (q @ q)
        x += alpha * p
        r -= alpha * q
        s = rmv(r)
        gnew = s @ s
        p = s + (gnew / gamma) * p
        gamma = gnew
        norms.append(np.linalg.norm(r))
    return x, np.array(norms)


def test_cgls_matches_numpy_on_oracle_operator_batched(problem):
    """The device CGLS (fm_cgls) with B = 4 columns at once: every column's
    iterate and residual history equal CGLS in NumPy on the oracle's stacked
    J / source-summed J^T, and the captured graph (8 iterations, replayed)
    gives the same bits as the eager iterations."""
    wl, states, ops = problem
    dev = torch.device("cuda:0")
    B, R, n_it = 4, wl.rcv.shape[0], 8
    A = _stacked_operator(wl, ops)
    mv, rmv = A.matvec, A.rmatvec
    d = np.random.default_rng(930).standard_normal((wl.S, R, B))
    d_dev = torch.from_numpy(d).to(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    batch = fm.Batch(states, B, fm.FM_FP64, stream=stream)
    cg = fm.Cgls(batch, max_iter=n_it)
    cg.start(d_dev)
    cg.iterate(n_it)
    batch.status()
    x_eager = cg.x().cpu().numpy()
    hist = np.sqrt(cg.history().cpu().numpy())
    for b in range(B):
        xr, nr = _cgls_numpy(mv, rmv, d[:, :, b].reshape(-1), n_it)
        assert np.linalg.norm(x_eager[:, b] - xr) <= 1e-9 * np.linalg.norm(xr), b
        assert np.allclose(hist[:, b], nr, rtol=1e-9, atol=0), b
        assert np.all(np.diff(hist[:, b]) <= 1e-12 * hist[0, b])
    cg.start(d_dev)
    cg.capture(n_it)
    for rep in range(3):
        cg.start(d_dev)
        cg.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cg.x().cpu().numpy(), x_eager), rep
        _ = torch.ones(10, device=dev).sum().item()     # eager work between replays
    cg.free()
    batch.free()
