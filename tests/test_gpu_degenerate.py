"""Degenerate grids on the GPU: the smallest grids the metric generator
makes (3 x 3, 3 x 3 x 3), a strip two cells deep (200 x 3) and a column
(3 x 3 x 40): levels of one node, workgroup shares that are empty for most
levels, sources in a corner of the grid.  Every mode against the oracle at
the FP64 bar, for the rhs-group kernel, node splits of 2 and 4 workgroups and
the balanced split, with the face stencil and with the 26-neighbour (cube)
stencil (8 neighbours in 2-D; on these grids most nodes lie on the boundary,
where components with an off-grid upstream neighbour are projected out)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import gpu_run, oracle_J, oracle_JT, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu

TOL64 = 1e-11

CASES = {
    "3x3": lambda: W.grids.deformed_2d(3, 3, 7001, 0.0, 0, S=1, B=16, R=2, name="3x3"),
    "strip 200x3": lambda: W.grids.deformed_2d(200, 3, 7002, 0.1, 1, S=2, B=16, R=7, name="strip 200x3"),
    "3x3x3": lambda: W.grids.deformed_3d(3, 3, 3, 7003, 1, 1, 16, 2, 2, name="3x3x3"),
    "column 3x3x40": lambda: W.grids.deformed_3d(3, 3, 40, 7004, 1, 1, 16, 1, 1, name="column 3x3x40"),
}
SCHEDULES = [{"split": 1}, {"split": 2}, {"split": 4}, {"balance": 3, "threads": 256, "unroll": 4}]
# the cube-stencil kernels are built for fewer shapes (256 threads: 3 nodes per thread)
SCHEDULES_CUBE = [{"split": 1}, {"split": 2}, {"split": 4}, {"balance": 3, "threads": 256, "unroll": 3}]


@pytest.mark.parametrize("stencil", [6, 26])
@pytest.mark.parametrize("case", list(CASES))
def test_degenerate_grids_all_modes(case, stencil):
    wl = CASES[case]()
    W.eikonal(wl)
    wl.stencil = stencil
    states, ops = states_for(fm, wl), oracle_ops(wl)
    B, R = 16, wl.rcv.shape[0]
    ds = seeded_ds(wl, B, 7100)
    p = seeded_ds(wl, B, 7101, per_pair=False)
    w = np.random.default_rng(7102).standard_normal((wl.S, wl.N, B))
    y = np.random.default_rng(7103).standard_normal((wl.S, R, B))
    refs = (oracle_J(ops, ds, True), oracle_J(ops, p, False, out="receivers"), oracle_JT(ops, w),
            O.apply_JT_summed(ops, list(y), "receivers"))
    for tun in (SCHEDULES if stencil == 6 else SCHEDULES_CUBE):
        print(f"case {case} stencil {stencil} N={wl.N} S={wl.S} {tun}", flush=True)
        x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tun)
        assert rel_l2_pairs(x, refs[0]) <= TOL64
        xr = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tun)
        assert rel_l2_pairs(xr, refs[1]) <= TOL64
        g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tun)
        assert rel_l2_pairs(g, refs[2]) <= TOL64
        gs = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tun)
        assert rel_l2(gs, refs[3]) <= TOL64
