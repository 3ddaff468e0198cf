"""The node-split kernels: P workgroups share one source and all B
right-hand sides and meet at the end of every level (Section 4.1: the nodes
of a level are independent; Section 4.3: block right-hand sides, then the
block solve).

* every mode (nodes / receivers in, per-source / summed out, per-pair /
  broadcast) against the oracle at the FP64 bar, for several P;
* bit-identical to the rhs-group kernel where both sum in the same order
  (singletons; blocks with B not a multiple of 16); with B a multiple of 16
  the block products run on the matrix cores (four products per step), so
  there the bar is 1e-13 against the rhs-group kernel and bit-identity
  across every node-split schedule (a difference would mean a value read
  before it was written or a stale cache line);
* rows shorter than a cache line (FP64 B=8, FP32 B=16) and an output array
  that does not start on a cache line take the invalidating barrier; FP32
  against the oracle at 1e-4;
* the batch status reports no timed-out wait.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import gpu_run, oracle_J, oracle_JT, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4
TOL_SCHED = 1e-13    # node split vs rhs groups where the block sums differ in grouping


def _same(a, b, tol=TOL_SCHED):
    return rel_l2_pairs(a, b) <= tol


@pytest.fixture(scope="module")
def curved():
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    wl.rcv = np.array([wl.node(i, j, 0) for j in range(0, 41, 4) for i in range(0, 41, 4)]
                      + [wl.node(20, 20, 0)], dtype=np.int64)
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.fixture(scope="module")
def multi2d():
    wl = W.grids.deformed_2d(161, 81, 2024, 0.4, 5, S=6, B=16, R=40, name="c2-family 161x81")
    W.eikonal(wl)
    return wl, states_for(fm, wl), oracle_ops(wl)


def test_tuning_reports_split(curved):
    wl, states, ops = curved
    b = fm.Batch(states, 16, fm.FM_FP64)
    assert b.tuning()["split"] > 1
    b.free()
    b = fm.Batch(states, 16, fm.FM_FP64, tuning={"split": 1})
    assert b.tuning()["split"] == 1
    b.free()
    b = fm.Batch(states, 3, fm.FM_FP64)
    assert b.tuning()["split"] == 1     # rows of 3 values: no node-split kernel
    b.free()
    with pytest.raises(fm.FmError):
        fm.Batch(states, 3, fm.FM_FP64, tuning={"split": 4})
    with pytest.raises(fm.FmError):
        fm.Batch(states, 16, fm.FM_FP64, tuning={"split": 3})


@pytest.mark.parametrize("P", [2, 4, 8, 16])
def test_curved_all_modes_fp64(curved, P):
    wl, states, ops = curved
    B = 16
    R = wl.rcv.shape[0]
    print(f"case split curved 41x41x25 (6 SCCs) B={B} P={P}", flush=True)
    tun = {"split": P}
    ds = seeded_ds(wl, B, 500 + P)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= TOL64
    x1 = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, {"split": 1})
    assert _same(x, x1)
    p = seeded_ds(wl, B, 600 + P, per_pair=False)
    xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
    assert rel_l2_pairs(xr, oracle_J(ops, p, False, out="receivers")) <= TOL64
    w = np.random.default_rng(700 + P).standard_normal((1, wl.N, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
    assert rel_l2_pairs(g, oracle_JT(ops, w)) <= TOL64
    g1 = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, {"split": 1})
    assert _same(g, g1)
    y = np.random.default_rng(800 + P).standard_normal((1, R, B))
    gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
    assert rel_l2(gs, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL64
    a, b = float(np.sum(xr * y)), float(np.sum(p * gs))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12


def test_multisource_2d_summed(multi2d):
    wl, states, ops = multi2d
    B = 16
    print("case split c2-family 161x81 S=6 B=16", flush=True)
    p = seeded_ds(wl, B, 901, per_pair=False)
    xb = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS)
    assert rel_l2_pairs(xb, oracle_J(ops, p, False, out="receivers")) <= TOL64
    y = np.random.default_rng(902).standard_normal((wl.S, wl.rcv.shape[0], B))
    gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED)
    assert rel_l2(gs, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL64
    gs1 = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, {"split": 1})
    assert rel_l2(gs, gs1) <= TOL_SCHED


@pytest.mark.parametrize("prec,B", [("fp64", 8), ("fp32", 16), ("fp32", 32)])
def test_short_rows_and_fp32(curved, prec, B):
    wl, states, ops = curved
    print(f"case split curved {prec} B={B}", flush=True)
    pr = fm.FM_FP64 if prec == "fp64" else fm.FM_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    ds = seeded_ds(wl, B, 1000 + B)
    x = gpu_run(fm, torch, states, B, pr, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, {"split": 4})
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= tol
    x1 = gpu_run(fm, torch, states, B, pr, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, {"split": 1})
    exact = B % 16 != 0          # vector block path: same order as the rhs-group kernel
    tol_s = TOL_SCHED if prec == "fp64" else 1e-6
    assert np.array_equal(x, x1) if exact else _same(x, x1, tol_s)
    w = np.random.default_rng(1100 + B).standard_normal((1, wl.N, B))
    g = gpu_run(fm, torch, states, B, pr, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, {"split": 4})
    assert rel_l2_pairs(g, oracle_JT(ops, w)) <= tol
    g1 = gpu_run(fm, torch, states, B, pr, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, {"split": 1})
    assert np.array_equal(g, g1) if exact else _same(g, g1, tol_s)


def test_unaligned_node_output(curved):
    """J with nodal output writes X into the caller's array; one that starts
    16 bytes past a cache line makes two nodes share lines."""
    wl, states, ops = curved
    B = 16
    dev = torch.device("cuda:0")
    ds = seeded_ds(wl, B, 1200)
    batch = fm.Batch(states, B, fm.FM_FP64, tuning={"split": 4})
    buf = torch.full((wl.N * B + 2,), float("nan"), device=dev, dtype=torch.float64)
    out = buf[2:].view(1, wl.N, B)
    assert out.data_ptr() % 128 == 16
    batch.apply_J(torch.from_numpy(ds).to(dev), fm.FM_DS_PER_PAIR, out, fm.FM_OUT_NODES)
    batch.status()
    x = out.cpu().numpy()
    batch.free()
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= TOL64
    x4 = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, {"split": 4})
    assert np.array_equal(x, x4)


def test_split_schedules_bit_identical_b16(curved):
    """With 16 right-hand sides (matrix-core block products) every node-split
    schedule must give the same bits."""
    wl, states, ops = curved
    B = 16
    ds = seeded_ds(wl, B, 1400)
    w = np.random.default_rng(1401).standard_normal((1, wl.N, B))
    outs = []
    scheds = [{"split": p, "unroll": u} for p in (2, 4, 8, 16) for u in (2, 4)]
    scheds += [{"split": p, "threads": 256, "unroll": u} for p in (4, 8) for u in (3, 4)]
    for tun in scheds:
        print(f"schedule {tun}", flush=True)
        outs.append((gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun),
                     gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)))
    for x, g in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(g, outs[0][1])


def test_repeated_applies_reuse_counters(curved):
    """Counters restart at every launch: many applies in a row on one batch
    give the same bits."""
    wl, states, ops = curved
    B = 16
    dev = torch.device("cuda:0")
    batch = fm.Batch(states, B, fm.FM_FP64, tuning={"split": 8})
    ds = torch.from_numpy(seeded_ds(wl, B, 1300)).to(dev)
    outs = []
    for _ in range(5):
        o = torch.empty((1, wl.N, B), device=dev, dtype=torch.float64)
        batch.apply_J(ds, fm.FM_DS_PER_PAIR, o, fm.FM_OUT_NODES)
        g = torch.empty((1, wl.N, B), device=dev, dtype=torch.float64)
        batch.apply_JT(o, fm.FM_W_NODES, g, fm.FM_JT_PER_SOURCE)
        outs.append((o, g))
    batch.status()
    for o, g in outs[1:]:
        assert torch.equal(o, outs[0][0]) and torch.equal(g, outs[0][1])
    batch.free()


@pytest.mark.parametrize("tuning", [{"split": 8, "threads": 256, "unroll": 3},
                                    {"balance": 3, "threads": 256, "unroll": 3}], ids=["uniform", "balanced"])
def test_split_placement_report(multi2d, tuning):
    """fm_batch_split_info reports, per source, the XCDs its workgroups ran on
    in the last apply: a non-empty set of the 8 XCDs; the rhs-group kernel has
    no such report."""
    wl, states, ops = multi2d
    B = 16
    dev = torch.device("cuda:0")
    batch = fm.Batch(states, B, fm.FM_FP64, tuning=tuning)
    ds = torch.from_numpy(seeded_ds(wl, B, 1400)).to(dev)
    o = torch.empty((wl.S, wl.N, B), device=dev, dtype=torch.float64)
    batch.apply_J(ds, fm.FM_DS_PER_PAIR, o, fm.FM_OUT_NODES)
    batch.status()
    xm = batch.split_info().astype(np.int64) & 0xFFFFFFFF
    one = sum(1 for m in xm if bin(int(m)).count("1") == 1)
    print(f"  {tuning}: masks {[hex(int(m)) for m in xm]}, {one} of {wl.S} sources on one XCD", flush=True)
    assert xm.shape == (wl.S,) and np.all(xm != 0) and np.all(xm < 256)
    batch.free()
    b1 = fm.Batch(states, B, fm.FM_FP64, tuning={"split": 1})
    with pytest.raises(fm.FmError):
        b1.split_info()
    b1.free()


def test_autotune_picks_a_measured_schedule(curved, tmp_path):
    """The schedule search measures the rhs-group kernel and every node-split
    shape that fits, returns the fastest, and that schedule reproduces the
    oracle."""
    wl, states, ops = curved
    B = 16
    R = wl.rcv.shape[0]
    dev = torch.device("cuda:0")
    p = torch.from_numpy(seeded_ds(wl, B, 1500, per_pair=False)).to(dev)
    y = torch.from_numpy(np.random.default_rng(1501).standard_normal((1, R, B))).to(dev)
    d = torch.empty((1, R, B), device=dev, dtype=torch.float64)
    g = torch.empty((wl.N, B), device=dev, dtype=torch.float64)
    best, table = fm.autotune(states, B, fm.FM_FP64, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                              y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED, reps=2, cache=False)
    for t, ms in table:
        print(f"{t} {ms:.3f} ms", flush=True)
    assert any(t["split"] == 1 for t, _ in table)
    assert any(t["split"] > 1 for t, _ in table)
    assert min(ms for _, ms in table) == [ms for t, ms in table if t == best][0]
    # the on-disk cache: the first call searches and stores, the second
    # returns the stored schedule without measuring anything
    cache = str(tmp_path / "tune.txt")
    b1, t1 = fm.autotune(states, B, fm.FM_FP64, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                         y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED, reps=1, cache=cache)
    b2, t2 = fm.autotune(states, B, fm.FM_FP64, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                         y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED, reps=1, cache=cache)
    assert len(t1) > 1 and t2 == [] and b1 == b2
    # another batch shape is another key: it searches again
    _, t3 = fm.autotune(states, B, fm.FM_FP64, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                        y, fm.FM_W_RECEIVERS, torch.empty((1, wl.N, B), device=dev, dtype=torch.float64),
                        fm.FM_JT_PER_SOURCE, reps=1, cache=cache)
    assert len(t3) > 1
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p.cpu().numpy(), fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, best)
    assert rel_l2_pairs(x, oracle_J(ops, p.cpu().numpy(), False, out="receivers")) <= TOL64


@pytest.mark.parametrize("which", ["curved", "multi2d"])
def test_balanced_split_bit_identical(which, curved, multi2d):
    """A different number of workgroups per source (balance = 1) changes only
    who computes which node, not any node's sum: same bits as the uniform
    split, in every mode."""
    wl, states, ops = curved if which == "curved" else multi2d
    B, R = 16, wl.rcv.shape[0]
    bal = {"balance": 7, "threads": 256, "unroll": 4}
    uni = {"split": 4}
    b = fm.Batch(states, B, fm.FM_FP64, tuning=bal)
    t = b.tuning()
    assert t["balance"] == 7 and t["split"] >= 2
    with pytest.raises(fm.FmError):
        fm.Batch(states, B, fm.FM_FP64, tuning={"balance": 11, "threads": 256, "unroll": 4})
    b.free()
    print(f"case balanced split {which} S={wl.S}: {t}", flush=True)
    ds = seeded_ds(wl, B, 1500)
    p = seeded_ds(wl, B, 1501, per_pair=False)
    w = np.random.default_rng(1502).standard_normal((wl.S, wl.N, B))
    y = np.random.default_rng(1503).standard_normal((wl.S, R, B))
    runs = [("J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES), ("J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS),
            ("JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE), ("JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED)]
    for d, x, im, om in runs:
        a1 = gpu_run(fm, torch, states, B, fm.FM_FP64, d, x, im, om, bal)
        a2 = gpu_run(fm, torch, states, B, fm.FM_FP64, d, x, im, om, uni)
        assert np.array_equal(a1, a2), (d, im, om)
    assert rel_l2_pairs(gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, bal),
                        oracle_J(ops, ds, True)) <= TOL64
    # FP32 (four lanes per node, 64-byte rows): the same bits as its uniform split
    a1 = gpu_run(fm, torch, states, B, fm.FM_FP32, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, bal)
    a2 = gpu_run(fm, torch, states, B, fm.FM_FP32, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, uni)
    assert np.array_equal(a1, a2)
    a1 = gpu_run(fm, torch, states, B, fm.FM_FP32, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, bal)
    a2 = gpu_run(fm, torch, states, B, fm.FM_FP32, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, uni)
    assert np.array_equal(a1, a2)
