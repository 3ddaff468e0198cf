"""GPU parity of J and J^T (through the C ABI) against the CPU oracle.

Bars (FP64): relative l2 per (source, rhs) pair <= 1e-11 against the oracle's
direct solves; transpose pairing <J ds, w> = <ds, J^T w> <= 1e-12.  FP32
variant: <= 1e-4 against the FP64 oracle.  Cases cover a 2-D grid (c1), the
controlled SCC fixture of Section 5.2 (nontrivial blocks), a multi-source 2-D
grid with receivers, ragged right-hand-side counts, every schedule (results
must be bit-identical across schedules) and the scaling identity of
Section 3.2.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import (gpu_run, oracle_J, oracle_JT, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds,
                     states_for)

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4
TOL_ADJ = 1e-12


@pytest.fixture(scope="module")
def c1():
    wl = W.config("c1")
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.fixture(scope="module")
def curved():
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    wl.rcv = np.array([wl.node(i, j, 0) for j in range(0, 41, 5) for i in range(0, 41, 5)]
                      + [wl.node(20, 20, 0)], dtype=np.int64)
    return wl, states_for(fm, wl), oracle_ops(wl)


def _adjoint(Jd, w, ds, JTw):
    a = float(np.sum(Jd * w))
    b = float(np.sum(ds * JTw))
    return abs(a - b) / max(abs(a), abs(b))


def test_c1_J_and_JT_fp64(c1):
    wl, states, ops = c1
    print("case c1 81x41, S=1, B=1", flush=True)
    ds = seeded_ds(wl, 1, 1000)
    x = gpu_run(fm, torch, states, 1, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    ref = oracle_J(ops, ds, True, solver="dense")
    assert rel_l2_pairs(x, ref) <= TOL64
    w = np.random.default_rng(1001).standard_normal((1, wl.N, 1))
    g = gpu_run(fm, torch, states, 1, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
    gref = oracle_JT(ops, w, solver="dense")
    assert rel_l2_pairs(g, gref) <= TOL64
    assert _adjoint(x, w, ds, g) <= TOL_ADJ


def test_curved_scc_fixture_fp64(curved):
    wl, states, ops = curved
    print("case curved 41x41x25 (6 SCCs), S=1, B=8", flush=True)
    assert states[0].stats()["n_scc"] == 6
    B = 8
    ds = seeded_ds(wl, B, 7)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    ref = oracle_J(ops, ds, True)
    assert rel_l2_pairs(x, ref) <= TOL64
    w = np.random.default_rng(8).standard_normal((1, wl.N, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
    gref = oracle_JT(ops, w)
    assert rel_l2_pairs(g, gref) <= TOL64
    for b in range(B):
        assert _adjoint(x[..., b], w[..., b], ds[..., b], g[..., b]) <= TOL_ADJ


def test_curved_receivers_and_duplicates(curved):
    wl, states, ops = curved
    print("case curved receivers (duplicate receiver), B=4", flush=True)
    B = 4
    R = wl.rcv.shape[0]
    ds = seeded_ds(wl, B, 17)
    xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_RECEIVERS)
    ref = oracle_J(ops, ds, True, out="receivers")
    assert rel_l2_pairs(xr, ref) <= TOL64
    y = np.random.default_rng(18).standard_normal((1, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_PER_SOURCE)
    gref = oracle_JT(ops, y, "receivers")
    assert rel_l2_pairs(g, gref) <= TOL64
    assert _adjoint(xr, y, ds, g) <= TOL_ADJ


def test_scaling_identity_gpu(curved):
    """Section 3.2: ds = -s reproduces dT = -T exactly for the frozen operator."""
    wl, states, ops = curved
    ds = np.repeat(-wl.s[None, :, None], 2, axis=2)
    x = gpu_run(fm, torch, states, 2, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    for b in range(2):
        assert rel_l2(x[0, :, b], -wl.T[0]) <= 1e-13


@pytest.fixture(scope="module")
def multi2d():
    wl = W.grids.deformed_2d(161, 81, 2024, 0.4, 5, S=6, B=6, R=40, name="c2-family 161x81")
    W.eikonal(wl)
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.mark.parametrize("B,rg", [(6, 2), (3, 1), (5, 1)])
def test_multisource_2d_ragged_batches(multi2d, B, rg):
    wl, states, ops = multi2d
    print(f"case c2-family 161x81 S=6 B={B} rg={rg}", flush=True)
    ds = seeded_ds(wl, B, 200 + B)
    tun = {"rhs_per_group": rg}
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
    ref = oracle_J(ops, ds, True)
    assert rel_l2_pairs(x, ref) <= TOL64
    p = seeded_ds(wl, B, 300 + B, per_pair=False)
    xb = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
    refb = oracle_J(ops, p, False, out="receivers")
    assert rel_l2_pairs(xb, refb) <= TOL64
    y = np.random.default_rng(400 + B).standard_normal((wl.S, wl.rcv.shape[0], B))
    gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
    gref = O.apply_JT_summed(ops, list(y), "receivers")
    assert rel_l2(gs, gref) <= TOL64
    # the pairing of the stacked J with the summed transpose (Section 4.4)
    a = float(np.sum(xb * y))
    b = float(np.sum(p * gs))
    assert abs(a - b) / max(abs(a), abs(b)) <= TOL_ADJ


def test_schedules_are_bit_identical(curved):
    """Each node's sum runs in a fixed order whatever the schedule, so every
    schedule must give the same bits; a difference would mean a value was read
    before it was written.  The schedules cover the rhs-group kernel and the
    node split (several workgroups per source meeting at every level)."""
    wl, states, ops = curved
    B = 8
    ds = seeded_ds(wl, B, 33)
    w = np.random.default_rng(34).standard_normal((1, wl.N, B))
    outs_J, outs_T = [], []
    schedules = [{"rhs_per_group": rg, "threads": nt, "xcd_aware": xcd, "split": 1}
                 for rg in (1, 2, 4, 8) for nt in (256, 1024) for xcd in (1, -1)]
    schedules += [{"split": p, "unroll": u} for p in (2, 4, 8, 16) for u in (2, 3, 4)]
    schedules += [{"split": p, "threads": 256, "unroll": 4} for p in (4, 8)]
    for tun in schedules:
        print(f"schedule {tun}", flush=True)
        outs_J.append(gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun))
        outs_T.append(gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun))
    for o in outs_J[1:]:
        assert np.array_equal(o, outs_J[0])
    for o in outs_T[1:]:
        assert np.array_equal(o, outs_T[0])


def test_fp32_variant(curved, multi2d):
    for wl, states, ops in (curved, multi2d):
        B = 4
        print(f"case fp32 {wl.name} B={B}", flush=True)
        ds = seeded_ds(wl, B, 55)
        x = gpu_run(fm, torch, states, B, fm.FM_FP32, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
        ref = oracle_J(ops, ds, True)
        assert rel_l2_pairs(x, ref) <= TOL32
        w = np.random.default_rng(56).standard_normal((wl.S, wl.N, B))
        g = gpu_run(fm, torch, states, B, fm.FM_FP32, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
        gref = oracle_JT(ops, w)
        assert rel_l2_pairs(g, gref) <= TOL32


def test_apply_argument_errors(c1):
    wl, states, ops = c1
    batch = fm.Batch(states, 1, fm.FM_FP64)
    dev = torch.device("cuda:0")
    x = torch.zeros((1, wl.N, 1), device=dev, dtype=torch.float64)
    with pytest.raises(ValueError):
        batch.apply_J(x.float(), fm.FM_DS_PER_PAIR, x, fm.FM_OUT_NODES)
    with pytest.raises(fm.FmError):
        fm.binding._check(fm.load().fm_apply_J(batch._ptr, fm.binding.C.c_void_p(x.data_ptr()), 7,
                                               fm.binding.C.c_void_p(x.data_ptr()), 0))
    with pytest.raises(fm.FmError):
        fm.Batch(states, 3, fm.FM_FP64, tuning={"rhs_per_group": 2})
    batch.free()
    # empty batches: no states, no right-hand sides
    with pytest.raises(fm.FmError, match="at least one state"):
        fm.Batch([], 16, fm.FM_FP64)
    with pytest.raises(fm.FmError, match="B must be"):
        fm.Batch(states, 0, fm.FM_FP64)
    # states without receivers: node outputs work, receiver modes are refused
    bare = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src)
    b0 = fm.Batch(bare, 1, fm.FM_FP64)
    assert b0.R == 0
    b0.apply_J(x, fm.FM_DS_PER_PAIR, x.clone(), fm.FM_OUT_NODES)
    b0.status()
    y = x.clone()
    with pytest.raises(fm.FmError, match="no receivers"):
        fm.binding._check(fm.load().fm_apply_J(b0._ptr, fm.binding.C.c_void_p(x.data_ptr()), fm.FM_DS_PER_PAIR,
                                               fm.binding.C.c_void_p(y.data_ptr()), fm.FM_OUT_RECEIVERS))
    b0.free()


def _sweep_run(states, B, direction, inp, in_mode, out_mode):
    dev = torch.device("cuda:0")
    batch = fm.Batch(states, B, fm.FM_FP64)
    S, N, R = batch.S, batch.N, batch.R
    x = torch.from_numpy(np.ascontiguousarray(inp)).to(dev)
    if direction == "J":
        out = torch.full((S, N, B) if out_mode == fm.FM_OUT_NODES else (S, R, B), float("nan"),
                         device=dev, dtype=torch.float64)
        cyc = batch.apply_J_sweep(x, in_mode, out, out_mode, want_cycles=True)
    else:
        out = torch.full((S, N, B) if out_mode == fm.FM_JT_PER_SOURCE else (N, B), float("nan"),
                         device=dev, dtype=torch.float64)
        cyc = batch.apply_JT_sweep(x, out, out_mode, want_cycles=True)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    batch.free()
    return res, cyc


@pytest.mark.parametrize("case", ["c1", "curved"])
def test_sweeping_baseline_matches_oracle(case, c1, curved):
    """The comparison baseline (directional Gauss-Seidel, Section 3.6) must
    reach the same frozen-operator answer as the oracle before any timing
    comparison means anything."""
    wl, states, ops = c1 if case == "c1" else curved
    B = 2
    print(f"case sweeping baseline {case} B={B}", flush=True)
    ds = seeded_ds(wl, B, 71)
    x, cyc = _sweep_run(states, B, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    assert np.all(cyc > 0), cyc
    ref = oracle_J(ops, ds, True)
    assert rel_l2_pairs(x, ref) <= TOL64
    w = np.random.default_rng(72).standard_normal((wl.S, wl.N, B))
    g, cyc2 = _sweep_run(states, B, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
    assert np.all(cyc2 > 0), cyc2
    gref = oracle_JT(ops, w)
    assert rel_l2_pairs(g, gref) <= TOL64
