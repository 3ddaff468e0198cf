"""The C-ABI library on the CPU (no GPU calls): it loads, exports every symbol
include/fmbtf.h declares, and its host setup (Algorithm 1, Phase I) matches
the oracle's explicit assembly, SCC partition, condensation levels and
structural statistics; invalid inputs and a singular SCC block are reported.
"""
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import diag
from oracle.assembly import assemble_workload

fm = pytest.importorskip("paper_2609_14982_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "fmbtf.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(fm_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 13
    lib = fm.load()
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert set(fm.binding.SYMBOLS) == declared


def _state(wl, a=0):
    return fm.build_frozen_state(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[a], wl.s, int(wl.src[a]), wl.rcv,
                                 stencil=getattr(wl, "stencil", 6))


def _compare_operator(wl, a=0):
    st = _state(wl, a)
    op = assemble_workload(wl, a)
    rowptr, col, w, c = st.export_operator()
    Wo = op.W.tocsr()
    Wo.sort_indices()
    assert np.array_equal(rowptr, Wo.indptr)
    assert np.array_equal(col, Wo.indices)
    # same FP64 formula in the same order: identical bits
    assert np.array_equal(w, Wo.data)
    assert np.array_equal(c, op.c)
    return st, op


def _compare_graph(st, op, T):
    comp, lf, lr = st.export_graph()
    ncomp, lab = diag.scc_labels(op.W)
    # same partition: a bijection between labels
    pairs = np.unique(np.stack([comp, lab], axis=1), axis=0)
    assert pairs.shape[0] == ncomp == len(np.unique(comp))
    olab, oclev, onlev = diag.condensation_levels(op.W)
    assert np.array_equal(lf, onlev)
    # reverse levels: longest path to a sink = levels of the transposed graph
    olab_r, _, onlev_r = diag.condensation_levels(op.W.T.tocsr())
    assert np.array_equal(lr, onlev_r)
    # component ids follow a topological order of the condensation DAG
    j, i = diag.edges(op.W)
    cross = comp[j] != comp[i]
    assert np.all(comp[j][cross] < comp[i][cross])
    fr = diag.fractions(op.W, T)
    s = st.stats()
    assert s["N"] == fr["N"] and s["E"] == fr["E"]
    assert s["n_scc"] == fr["n_scc"] and s["n_cyc"] == fr["n_cyc"]
    assert s["largest_scc"] == fr["largest_scc"]
    assert s["n_vio"] == fr["n_vio"] and s["n_unr"] == fr["n_unr"]
    assert s["levels_fwd"] == onlev.max() + 1
    assert s["levels_rev"] == onlev_r.max() + 1


def test_setup_matches_oracle_c1():
    wl = W.config("c1")
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])


@pytest.mark.parametrize("n", [(21, 21, 13), (41, 41, 25)])
def test_setup_matches_oracle_curved_scc(n):
    wl = W.curved_state(*n, A=500.0, eps_T=0.05)
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])
    assert st.stats()["n_scc"] > 0


def test_setup_matches_oracle_manufactured():
    wl, _, _ = W.manufactured(21, 21, 11)
    st, op = _compare_operator(wl)
    _compare_graph(st, op, wl.T[0])


@pytest.mark.slow
def test_setup_matches_oracle_c3_one_source():
    wl = W.config("c3")
    st, op = _compare_operator(wl, 3)
    _compare_graph(st, op, wl.T[3])


def test_multi_source_build_matches_single():
    wl = W.grids.deformed_2d(61, 31, 77, 0.4, 2, S=3, B=2, R=12, name="mini")
    W.eikonal(wl)
    many = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src, wl.rcv,
                                  nthreads=3)
    for a, st in enumerate(many):
        one = _state(wl, a)
        s1, s2 = one.stats(), st.stats()
        s1.pop("setup_seconds"), s2.pop("setup_seconds")
        assert s1 == s2
        for x, y in zip(one.export_operator(), st.export_operator()):
            assert np.array_equal(x, y)


def _expect_error(code, **kw):
    wl = W.config("c1")
    args = dict(dim=2, n1=wl.n1, n2=1, n3=wl.n3, G=wl.G, T=wl.T[0], s=wl.s, src_node=int(wl.src[0]),
                rcv_nodes=wl.rcv)
    args.update(kw)
    with pytest.raises(fm.FmError) as ei:
        fm.build_frozen_state(**args)
    assert ei.value.code == code
    return str(ei.value)


def test_invalid_inputs_are_rejected():
    wl = W.config("c1")
    T_bad = wl.T[0].copy()
    T_bad[int(wl.src[0])] = 1e-3
    assert "source" in _expect_error(fm.binding.FM_EINVAL, T=T_bad)
    s_bad = wl.s.copy()
    s_bad[7] = 0.0
    _expect_error(fm.binding.FM_EINVAL, s=s_bad)
    s_nan = wl.s.copy()
    s_nan[9] = np.nan
    _expect_error(fm.binding.FM_EINVAL, s=s_nan)
    T_inf = wl.T[0].copy()
    T_inf[11] = np.inf
    _expect_error(fm.binding.FM_EINVAL, T=T_inf)
    _expect_error(fm.binding.FM_EINVAL, src_node=wl.N)
    _expect_error(fm.binding.FM_EINVAL, src_node=-1)
    _expect_error(fm.binding.FM_EINVAL, rcv_nodes=np.array([0, wl.N + 3]))
    _expect_error(fm.binding.FM_EINVAL, dim=4)
    _expect_error(fm.binding.FM_EINVAL, n2=2)


def test_singular_scc_block_is_reported():
    """Section 4.2: a closed SCC whose rows take all their weight from inside
    the component (every internal row sum is 1) violates the hypotheses of
    Theorem 1; its block I - W_CC is singular and the setup must say so.
    The 3 x 3 input below has such a component on nodes {4, 5, 7, 8}; the
    oracle confirms the closed component and the zero determinant."""
    G = np.tile([1.0, 1.0, 0.65], (9, 1))
    T = np.array([0.0, 3.9, 3.4, 0.8, 0.5, 1.1, 1.8, 0.9, 0.9])
    s = np.ones(9)
    op = O.assemble(2, 3, 1, 3, G, T, s, 0)
    comps = diag.scc_summary(op.W)
    assert [c.tolist() for c in comps] == [[4, 5, 7, 8]]
    Wcc = op.W[comps[0]][:, comps[0]].toarray()
    assert np.allclose(Wcc.sum(axis=1), 1.0)
    with pytest.raises(fm.FmError) as ei:
        fm.build_frozen_state(2, 3, 1, 3, G, T, s, 0)
    assert ei.value.code == fm.binding.FM_ESINGULAR
    assert "4 nodes" in str(ei.value)


def test_block_inverse_residuals_are_recorded():
    """Section 4.3 factors every block with pivoting; the setup also checks
    the stored inverse, ||A_C X e_j - e_j||_inf on four columns, and records
    the largest value in the statistics (0 when no block keeps an inverse)."""
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    st = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src)[0].stats()
    assert st["n_scc"] == 6 and 0.0 < st["block_residual"] <= 1e-13
    flat = W.config("c1")
    st = fm.build_frozen_states(flat.dim, flat.n1, flat.n2, flat.n3, flat.G, flat.T, flat.s, flat.src)[0].stats()
    if st["n_scc"] == 0:
        assert st["block_residual"] == 0.0
