"""The 26-neighbour (cube) stencil through the C ABI on the CPU (no GPU
calls): the host setup's W and c are bit-identical to the oracle's cube
assembly (same FP64 operations in the same order), and its SCC partition,
condensation levels and structural statistics match the oracle's graph
diagnostics, on 2-D and 3-D deformed grids, the curved-wavefront fixture and
c3, on degenerate grids (3 x 3, a 200 x 3 strip, 3 x 3 x 3, a 3 x 3 x 40
column), and with an off-grid point source (identity seed rows); an unknown
stencil value is rejected.
"""
import numpy as np
import pytest

import workloads as W
from test_abi_cpu import _compare_graph, _compare_operator

fm = pytest.importorskip("paper_2609_14982_amd")


def _cube(wl):
    wl.stencil = 26
    return wl


def test_cube_setup_matches_oracle_c1():
    wl = _cube(W.config("c1"))
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])
    # dependencies beyond the faces occur (corner neighbours in 2-D)
    rowptr, col, _, _ = st.export_operator()
    rows = np.repeat(np.arange(wl.N), np.diff(rowptr))
    d = np.abs(col - rows)
    assert np.any((d != 1) & (d != wl.n1))


@pytest.mark.parametrize("n", [(21, 21, 13), (41, 41, 25)])
def test_cube_setup_matches_oracle_curved(n):
    wl = _cube(W.curved_state(*n, A=500.0, eps_T=0.05))
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])
    print("cube stencil, curved", n, {k: st.stats()[k] for k in ("E", "n_scc", "largest_scc", "levels_fwd")})


def test_cube_setup_matches_oracle_deformed_3d():
    wl = _cube(W.smooth_3d(25, 23, 13, topo_amp=0.2))
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])


@pytest.mark.parametrize("case", ["3x3", "strip", "3x3x3", "column"])
def test_cube_setup_matches_oracle_degenerate(case):
    """The smallest grids and a strip and column a few nodes wide: most nodes
    are boundary nodes, so most rows take the projected (one-sided) form."""
    make = {
        "3x3": lambda: W.grids.deformed_2d(3, 3, 7001, 0.0, 0, S=1, B=16, R=2, name="3x3"),
        "strip": lambda: W.grids.deformed_2d(200, 3, 7002, 0.1, 1, S=2, B=16, R=7, name="strip 200x3"),
        "3x3x3": lambda: W.grids.deformed_3d(3, 3, 3, 7003, 1, 1, 16, 2, 2, name="3x3x3"),
        "column": lambda: W.grids.deformed_3d(3, 3, 40, 7004, 1, 1, 16, 1, 1, name="column 3x3x40"),
    }
    wl = make[case]()
    W.eikonal(wl)
    _cube(wl)
    for a in range(wl.S):
        st, op = _compare_operator(wl, a)
        _compare_graph(st, op, wl.T[a])


@pytest.mark.slow
def test_cube_setup_matches_oracle_c3_one_source():
    wl = _cube(W.config("c3"))
    st, op = _compare_operator(wl, 3)
    _compare_graph(st, op, wl.T[3])
    print("cube stencil, c3 source 3", st.stats())


def test_unknown_stencil_is_rejected():
    wl = W.config("c1")
    for bad in (5, 8, 27, -1):
        with pytest.raises(fm.FmError) as e:
            fm.build_frozen_state(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[0], wl.s, int(wl.src[0]), wl.rcv,
                                  stencil=bad)
        assert e.value.code == fm.binding.FM_EINVAL and "stencil" in str(e.value)


def test_cube_point_source_matches_oracle():
    from oracle import source as PS
    wl = W.smooth_3d(17, 15, 9, topo_amp=0.1, with_T=False)
    xi = np.array([[6.3, 7.1, 0.0], [11.6, 3.2, 2.5]])
    W.eikonal_point(wl, xi, 1.5)
    states = fm.build_frozen_states_pt(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, wl.T, wl.s, xi, 1.5, wl.rcv, stencil=26)
    for a in range(2):
        pso = PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, wl.T[a], wl.s, xi[a], 1.5, wl.rcv,
                                       stencil=26)
        rowptr, col, wv, c = states[a].export_operator()
        Wo = pso.op.W.tocsr()
        Wo.sort_indices()
        assert np.array_equal(rowptr, Wo.indptr) and np.array_equal(col, Wo.indices)
        assert np.array_equal(wv, Wo.data)
        c_ref = pso.op.c.copy()
        c_ref[pso.seeds] = 0.0
        assert np.array_equal(c, c_ref)
        assert states[a].stats()["n_seed"] == pso.seeds.size
