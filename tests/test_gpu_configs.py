"""Parity of the remaining benchmark configurations against the oracle:

* c2 (401 x 201 2-D deformed grid, 16 sources x 32 rhs, 100 receivers),
  FP64 (the node split with 16 lanes per node, and the rhs-group kernel) and
  FP32 (the node split, four values per 16-byte lane access): J from a
  broadcast model block to
  receivers and the source-summed J^T from receiver data, against SuperLU
  solves of the explicit operator (FP64 bar 1e-11, FP32 bar 1e-4), and the
  transpose pairing;
* c3 (101 x 101 x 51 3-D deformed grid, 8 sources x 16 rhs, 100 receivers),
  FP64 node split: per-pair J at every node and the per-source J^T on
  sampled sources against the oracle's converged Gauss-Seidel sweeping, and
  the pairing of the stacked J with the summed J^T over all sources.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import gpu_run, oracle_J, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for
from oracle.assembly import assemble_workload

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL64 = 1e-11
TOL32 = 1e-4
TOL_ADJ = 1e-12


@pytest.fixture(scope="module")
def c2():
    print("case c2 401x201, S=16, B=32: building", flush=True)
    wl = W.config("c2")
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.fixture(scope="module")
def c3():
    print("case c3 101x101x51, S=8, B=16: building", flush=True)
    wl = W.config("c3")
    return wl, states_for(fm, wl)


def _pairing(d, y, p, g):
    a = float(np.sum(d * y))
    b = float(np.sum(p * g))
    return abs(a - b) / max(abs(a), abs(b))


@pytest.mark.parametrize("prec,tuning", [("fp64", None), ("fp32", None), ("fp64", {"split": 1}),
                                         ("fp64", {"split": 4, "threads": 256, "unroll": 3}),
                                         ("fp64", {"split": 8, "threads": 256, "unroll": 2})])
def test_c2_receivers_and_source_sum(c2, prec, tuning):
    """c2's 32 rhs: FP64 rows of 256 bytes take the node split with 16 lanes
    per node (the library's choice) as well as the rhs-group kernel; FP32
    rows of 128 bytes take 8 lanes per node."""
    wl, states, ops = c2
    B, R = wl.B, wl.rcv.shape[0]
    pr = fm.FM_FP64 if prec == "fp64" else fm.FM_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    b = fm.Batch(states, B, pr, tuning=tuning)
    used = b.tuning()
    print(f"c2 {prec} schedule {used}", flush=True)
    b.free()
    if tuning is None or tuning.get("split", 1) > 1:
        assert used["split"] > 1
    p = seeded_ds(wl, B, 2100, per_pair=False)
    d = gpu_run(fm, torch, states, B, pr, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tuning)
    assert rel_l2_pairs(d, oracle_J(ops, p, False, out="receivers")) <= tol
    y = np.random.default_rng(2101).standard_normal((wl.S, R, B))
    g = gpu_run(fm, torch, states, B, pr, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tuning)
    assert rel_l2(g, O.apply_JT_summed(ops, list(y), "receivers")) <= tol
    if prec == "fp64":
        for k in range(B):
            assert _pairing(d[..., k], y[..., k], p[:, k], g[:, k]) <= TOL_ADJ


def test_c3_split_sampled_sources_and_pairing(c3):
    wl, states = c3
    S, B, R = wl.S, wl.B, wl.rcv.shape[0]
    b = fm.Batch(states, B, fm.FM_FP64)
    print(f"c3 schedule {b.tuning()}", flush=True)
    assert b.tuning()["split"] > 1
    b.free()
    ds = seeded_ds(wl, B, 3100)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    w = np.random.default_rng(3101).standard_normal((S, wl.N, B))
    gps = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
    threads = min(16, os.cpu_count() or 1)
    for a in (0, S // 2, S - 1):
        print(f"oracle source {a}", flush=True)
        op = assemble_workload(wl, a)
        xo = O.gs_solve(op, op.W, op.c[:, None] * ds[a], nthreads=threads)
        assert rel_l2_pairs(x[a:a + 1], xo[None]) <= TOL64
        lam = O.gs_solve(op, op.WT(), w[a], nthreads=threads)
        assert rel_l2_pairs(gps[a:a + 1], (op.c[:, None] * lam)[None]) <= TOL64
    p = seeded_ds(wl, B, 3102, per_pair=False)
    d = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS)
    y = np.random.default_rng(3103).standard_normal((S, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED)
    for k in range(B):
        assert _pairing(d[..., k], y[..., k], p[:, k], g[:, k]) <= TOL_ADJ
