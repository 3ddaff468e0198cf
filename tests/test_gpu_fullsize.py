"""Parity at the benchmark's full size: the 201 x 201 x 101 deformed grid,
64 sources x 16 right-hand sides, 400 receivers, in the launch configuration
bench.py times (default schedule, FP64).

The oracle cannot solve all 1,024 systems quickly, so:
* sampled sources (fewest, median and most SCC entries, i.e. the largest
  blocks) are compared with the oracle's converged Gauss-Seidel sweeping
  (explicit assembly, plain C) - every node and every receiver, J and J^T;
* properties that hold at any size are checked on all sources: the transpose
  pairing of the stacked J with the source-summed J^T (Section 4.4), and the
  equality of the summed transpose with the sum of per-source transposes.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import rel_l2_pairs
from oracle.assembly import assemble_workload

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL64 = 1e-11
TOL_ADJ = 1e-12


@pytest.fixture(scope="module")
def c4():
    print("case c4 201x201x101, S=64, B=16: building", flush=True)
    wl = W.config("c4")
    states = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src, wl.rcv)
    k2 = np.array([s.stats()["sum_k2"] for s in states])
    order = np.argsort(k2)
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    print(f"sampled sources {sample}, sum k^2 {k2[sample].tolist()}", flush=True)
    return wl, states, sample


def _oracle_nodes(wl, a, q, transpose):
    op = assemble_workload(wl, a)
    threads = min(16, os.cpu_count() or 1)
    if transpose:
        lam = O.gs_solve(op, op.WT(), q, nthreads=threads)
        return op, op.c[:, None] * lam
    x = O.gs_solve(op, op.W, op.c[:, None] * q, nthreads=threads)
    return op, x


def test_c4_sampled_sources_match_oracle(c4):
    wl, states, sample = c4
    B = wl.B
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4100)
    p = W.smooth_noise(wl, B, rng)
    y = rng.standard_normal((len(sample), wl.rcv.shape[0], B))
    sub = [states[a] for a in sample]
    batch = fm.Batch(sub, B, fm.FM_FP64)
    S = len(sample)
    d_p = torch.from_numpy(p).to(dev)
    xn = torch.empty((S, wl.N, B), dtype=torch.float64, device=dev)
    xr = torch.empty((S, wl.rcv.shape[0], B), dtype=torch.float64, device=dev)
    gn = torch.empty((S, wl.N, B), dtype=torch.float64, device=dev)
    batch.apply_J(d_p, fm.FM_DS_BROADCAST, xn, fm.FM_OUT_NODES)
    batch.apply_J(d_p, fm.FM_DS_BROADCAST, xr, fm.FM_OUT_RECEIVERS)
    batch.apply_JT(torch.from_numpy(y).to(dev), fm.FM_W_RECEIVERS, gn, fm.FM_JT_PER_SOURCE)
    torch.cuda.synchronize()
    xn, xr, gn = xn.cpu().numpy(), xr.cpu().numpy(), gn.cpu().numpy()
    batch.free()
    for i, a in enumerate(sample):
        print(f"oracle source {a}", flush=True)
        op, xo = _oracle_nodes(wl, a, p, False)
        assert rel_l2_pairs(xn[i:i + 1], xo[None]) <= TOL64
        assert rel_l2_pairs(xr[i:i + 1], xo[None, wl.rcv]) <= TOL64
        r = O.solve.scatter_receivers(op, y[i])
        _, go = _oracle_nodes(wl, a, r, True)
        assert rel_l2_pairs(gn[i:i + 1], go[None]) <= TOL64


def test_c4_all_sources_pairing_and_source_sum(c4):
    wl, states, sample = c4
    B, S, R = wl.B, wl.S, wl.rcv.shape[0]
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(4200)
    batch = fm.Batch(states, B, fm.FM_FP64)
    p = torch.randn((wl.N, B), device=dev, dtype=torch.float64, generator=gen)
    y = torch.randn((S, R, B), device=dev, dtype=torch.float64, generator=gen)
    d = torch.empty((S, R, B), device=dev, dtype=torch.float64)
    g = torch.empty((wl.N, B), device=dev, dtype=torch.float64)
    batch.apply_J(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
    batch.apply_JT(y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
    torch.cuda.synchronize()
    for b in range(B):
        lhs = float(torch.sum(d[..., b] * y[..., b]))
        rhs = float(torch.sum(p[:, b] * g[:, b]))
        assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) <= TOL_ADJ, b
    # the summed transpose equals the sum of per-source transposes (fixed order)
    acc = torch.zeros_like(g)
    for a0 in range(0, S, 16):
        part = fm.Batch(states[a0:a0 + 16], B, fm.FM_FP64)
        gp = torch.empty((16, wl.N, B), device=dev, dtype=torch.float64)
        part.apply_JT(y[a0:a0 + 16].contiguous(), fm.FM_W_RECEIVERS, gp, fm.FM_JT_PER_SOURCE)
        for k in range(16):
            acc += gp[k]
        del gp
        part.free()
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(acc - g) / torch.linalg.norm(g))
    assert err <= 1e-14, err
    batch.free()
