"""Large SCC blocks solved by their Neumann series instead of a stored
inverse (Section 6 names iterative solvers for large components; Theorem 1
gives rho(W_CC) < 1): x_C = sum_{j<=m} W_CC^j b_C, m fixed at build time so
that ||W_CC^{m+1}||_inf <= 2^-56 (primal) and ||W_CC^{m+1}||_1 <= 2^-56
(transpose).

Host side (no GPU): the number of terms the library stores for every block
of the curved fixture equals the least m with that bound, computed here from
the oracle's explicit W; the operator and the structure statistics do not
depend on the block solver; the threshold setting is validated.

GPU: every block of the curved fixture (6 SCCs) and of three c3 sources
solved iteratively, against the oracle at 1e-11 in every mode, for the
rhs-group kernel and node splits of 2, 4, 8 workgroups (bit-identical to
each other: each row sums its couplings in one fixed order) and against the
dense-inverse solve at 1e-13; FP32 at 1e-4.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

import oracle as O
import workloads as W
from oracle.assembly import assemble_workload
from helpers import gpu_run, oracle_J, oracle_JT, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

TOL64 = 1e-11
TOL32 = 1e-4
TOL_DENSE = 1e-13


@pytest.fixture
def iterative_all():
    """States built inside this fixture solve every block iteratively."""
    fm.set_iterative_block_min(2)
    yield
    fm.set_iterative_block_min(0)


@pytest.fixture(scope="module")
def curved():
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    wl.rcv = np.array([wl.node(i, j, 0) for j in range(0, 41, 4) for i in range(0, 41, 4)]
                      + [wl.node(20, 20, 0)], dtype=np.int64)
    return wl, oracle_ops(wl)


def _terms(Wc):
    """Least m >= 1 with max(W^{m+1} 1) <= 2^-56 (W >= 0)."""
    v = np.ones(Wc.shape[0])
    for j in range(1, 202):
        v = Wc @ v
        if v.max() <= 2.0 ** -56:
            return max(j - 1, 1)
    return 0


def test_series_terms_match_the_bound(curved, iterative_all):
    wl, ops = curved
    st = states_for(fm, wl)[0]
    s = st.stats()
    Wm = ops[0].W.tocsr()
    ncomp, lab = cg.connected_components(Wm, directed=True, connection="strong")
    sizes = np.bincount(lab)
    blocks = [np.nonzero(lab == c)[0] for c in np.nonzero(sizes > 1)[0]]
    assert s["n_iter_blocks"] == len(blocks) == 6 and s["dense_k2"] == 0
    mf = [_terms(Wm[b][:, b]) for b in blocks]
    mr = [_terms(Wm[b][:, b].T.tocsr()) for b in blocks]
    assert min(mf + mr) >= 1
    assert s["max_iter"] == max(mf + mr)
    assert s["iter_nnz"] == sum(Wm[b][:, b].nnz for b in blocks)
    # the operator and the structure do not depend on the block solver
    fm.set_iterative_block_min(-1)
    dense = states_for(fm, wl)[0]
    for x, y in zip(dense.export_operator(), st.export_operator()):
        assert np.array_equal(x, y)
    d = dense.stats()
    assert d["n_iter_blocks"] == 0 and d["sum_k2"] == s["sum_k2"] == d["dense_k2"]
    for key in ("n_scc", "largest_scc", "levels_fwd", "levels_rev", "n_cyc"):
        assert d[key] == s[key]
    assert s["state_bytes"] < d["state_bytes"]


def test_threshold_argument():
    with pytest.raises(fm.FmError):
        fm.set_iterative_block_min(1)
    fm.set_iterative_block_min(0)


@pytest.mark.gpu
@pytest.mark.parametrize("tun", [{"split": 1}, {"split": 2}, {"split": 4}, {"split": 8}])
def test_curved_iterative_blocks_all_modes(curved, iterative_all, tun):
    wl, ops = curved
    B, R = 16, wl.rcv.shape[0]
    print(f"case iterative blocks curved 41x41x25 B={B} {tun}", flush=True)
    states = states_for(fm, wl)
    assert states[0].stats()["n_iter_blocks"] == 6
    ds = seeded_ds(wl, B, 3100)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= TOL64
    p = seeded_ds(wl, B, 3101, per_pair=False)
    xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
    assert rel_l2_pairs(xr, oracle_J(ops, p, False, out="receivers")) <= TOL64
    w = np.random.default_rng(3102).standard_normal((1, wl.N, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
    assert rel_l2_pairs(g, oracle_JT(ops, w)) <= TOL64
    y = np.random.default_rng(3103).standard_normal((1, R, B))
    gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
    assert rel_l2(gs, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL64
    a, b = float(np.sum(xr * y)), float(np.sum(p * gs))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12
    # against the dense-inverse solve of the same blocks
    fm.set_iterative_block_min(-1)
    dense = states_for(fm, wl)
    assert dense[0].stats()["n_iter_blocks"] == 0
    xd = gpu_run(fm, torch, dense, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
    gd = gpu_run(fm, torch, dense, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
    print(f"  iterative vs dense: J {rel_l2_pairs(x, xd):.2e}, J^T {rel_l2_pairs(g, gd):.2e}", flush=True)
    assert rel_l2_pairs(x, xd) <= TOL_DENSE and rel_l2_pairs(g, gd) <= TOL_DENSE


@pytest.mark.gpu
def test_iterative_blocks_bit_identical_across_splits(curved, iterative_all):
    wl, ops = curved
    B = 16
    print("case iterative blocks: node-split schedules bit-identical", flush=True)
    states = states_for(fm, wl)
    ds = seeded_ds(wl, B, 3200)
    w = np.random.default_rng(3201).standard_normal((1, wl.N, B))
    ref = None
    for tun in ({"split": 2}, {"split": 4}, {"split": 8}, {"split": 4, "threads": 256, "unroll": 3}):
        x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
        g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
        if ref is None:
            ref = (x, g)
        else:
            assert np.array_equal(ref[0], x) and np.array_equal(ref[1], g), tun


@pytest.mark.gpu
@pytest.mark.parametrize("prec,B,tun", [("fp64", 8, {"split": 4}), ("fp32", 16, {"split": 4}),
                                        ("fp32", 4, {"split": 1})])
def test_iterative_blocks_short_rows_and_fp32(curved, iterative_all, prec, B, tun):
    wl, ops = curved
    print(f"case iterative blocks curved {prec} B={B} {tun}", flush=True)
    states = states_for(fm, wl)
    pr = fm.FM_FP64 if prec == "fp64" else fm.FM_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    ds = seeded_ds(wl, B, 3300 + B)
    x = gpu_run(fm, torch, states, B, pr, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= tol
    w = np.random.default_rng(3400 + B).standard_normal((1, wl.N, B))
    g = gpu_run(fm, torch, states, B, pr, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
    assert rel_l2_pairs(g, oracle_JT(ops, w)) <= tol


@pytest.mark.gpu
def test_c3_iterative(iterative_all):
    """c3 (101 x 101 x 51, blocks up to 693 nodes): three sources, every
    block iterative, against the oracle's converged Gauss-Seidel sweeping
    (SuperLU does not finish on this grid in minutes)."""
    wl = W.config("c3")
    S, B, R = 3, wl.B, wl.rcv.shape[0]
    print(f"case iterative blocks c3 101x101x51 S={S} B={B}", flush=True)
    states = states_for(fm, wl, S)
    n_it = sum(s.stats()["n_iter_blocks"] for s in states)
    n_blk = sum(s.stats()["n_scc"] for s in states)
    print(f"  {n_blk} blocks, all iterative; most terms {max(s.stats()['max_iter'] for s in states)}", flush=True)
    assert n_it == n_blk > 0
    p = seeded_ds(wl, B, 3500, per_pair=False)
    xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS)
    y = np.random.default_rng(3501).standard_normal((S, R, B))
    gp = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_PER_SOURCE)
    print("  gpu done", flush=True)
    threads = min(16, os.cpu_count() or 1)
    for a in range(S):
        print(f"  oracle source {a}", flush=True)
        op = assemble_workload(wl, a)
        x = O.gs_solve(op, op.W, op.c[:, None] * p, nthreads=threads)
        assert rel_l2_pairs(xr[a:a + 1], (op.P() @ x)[None]) <= TOL64
        lam = O.gs_solve(op, op.WT(), O.solve.scatter_receivers(op, y[a]), nthreads=threads)
        assert rel_l2_pairs(gp[a:a + 1], (op.c[:, None] * lam)[None]) <= TOL64
