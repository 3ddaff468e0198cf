"""Interpolating receivers on the GPU: P_alpha of Section 4.4 as weighted
entries over a few nodes per receiver (bilinear on the 3-D surface, linear on
the 2-D one), in the primal gather and in the transpose's receiver scatter.

* J to receivers and J^T from receivers (per source and summed) against the
  oracle's explicit sampling matrix, FP64 at 1e-11 and FP32 at 1e-4, for the
  rhs-group kernel and node splits of 2 and 4 workgroups;
* a source's weighted entries either staged in LDS (240 entries) or read from
  global memory (1,200 entries, beyond the 64 KB staging area);
* the adjoint pairing <J p, y> = <p, J^T y> at 1e-12;
* one entry of weight 1 per receiver gives the same bits as the plain
  selection.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import gpu_run, oracle_J, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4


def _with_receivers(wl, R, seed):
    nodes, w, _ = W.interpolating_receivers(wl, R, seed)
    wl.rcv, wl.rcv_w = nodes, w
    return wl


@pytest.fixture(scope="module")
def grid3d():
    wl = W.grids.deformed_3d(41, 37, 21, 4100, 2, 2, 16, 1, 1, name="rcv-3d 41x37x21")
    W.eikonal(wl)
    return wl


@pytest.fixture(scope="module", params=[60, 300], ids=["lds", "global"])
def interp3d(request, grid3d):
    import copy
    wl = _with_receivers(copy.copy(grid3d), request.param, 4200 + request.param)
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.fixture(scope="module")
def interp2d():
    wl = W.grids.deformed_2d(161, 81, 4300, 0.4, 3, S=3, B=16, R=10, name="rcv-2d 161x81")
    W.eikonal(wl)
    wl = _with_receivers(wl, 25, 4301)
    return wl, states_for(fm, wl), oracle_ops(wl)


@pytest.mark.parametrize("tun", [{"split": 1}, {"split": 2}, {"split": 4}], ids=["groups", "P2", "P4"])
def test_interpolating_receivers_fp64(interp3d, tun):
    wl, states, ops = interp3d
    B, R = 16, wl.rcv.shape[0]
    print(f"case receivers 3-D R={R} K=4 {tun}", flush=True)
    p = seeded_ds(wl, B, 4400, per_pair=False)
    xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
    assert rel_l2_pairs(xr, oracle_J(ops, p, False, out="receivers")) <= TOL64
    y = np.random.default_rng(4401).standard_normal((wl.S, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_PER_SOURCE, tun)
    gref = np.stack([O.apply_JT(op, y[a], "receivers") for a, op in enumerate(ops)])
    assert rel_l2_pairs(g, gref) <= TOL64
    gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
    assert rel_l2(gs, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL64
    a, b = float(np.sum(xr * y)), float(np.sum(p * gs))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12


def test_interpolating_receivers_2d_and_fp32(interp2d):
    wl, states, ops = interp2d
    B, R = 16, wl.rcv.shape[0]
    for prec, tol in ((fm.FM_FP64, TOL64), (fm.FM_FP32, TOL32)):
        print(f"case receivers 2-D R={R} K=2 precision {prec}", flush=True)
        p = seeded_ds(wl, B, 4500, per_pair=False)
        xr = gpu_run(fm, torch, states, B, prec, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS)
        assert rel_l2_pairs(xr, oracle_J(ops, p, False, out="receivers")) <= tol
        y = np.random.default_rng(4501).standard_normal((wl.S, R, B))
        gs = gpu_run(fm, torch, states, B, prec, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED)
        assert rel_l2(gs, O.apply_JT_summed(ops, list(y), "receivers")) <= tol


def test_unit_weights_equal_the_selection(grid3d):
    import copy
    wl = copy.copy(grid3d)
    sel = np.array([wl.node(i, j, 0) for j in range(0, 37, 6) for i in range(0, 41, 5)], dtype=np.int64)
    wl.rcv, wl.rcv_w = sel, None
    plain = states_for(fm, wl)
    wl.rcv, wl.rcv_w = sel[:, None], np.ones((sel.shape[0], 1))
    unit = states_for(fm, wl)
    B, R = 16, sel.shape[0]
    print(f"case receivers unit weights R={R}", flush=True)
    p = seeded_ds(wl, B, 4600, per_pair=False)
    y = np.random.default_rng(4601).standard_normal((wl.S, R, B))
    for tun in ({"split": 1}, {"split": 4}):
        a = gpu_run(fm, torch, plain, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
        b = gpu_run(fm, torch, unit, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
        assert np.array_equal(a, b)
        a = gpu_run(fm, torch, plain, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
        b = gpu_run(fm, torch, unit, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
        assert np.array_equal(a, b)
