"""Pins of the oracle's graph diagnostics (no GPU).

* SCCs (Section 4.1) against brute-force mutual reachability on random digraphs.
* Proposition 2 (Section 3.5): the Kahn residual is exactly the set of vertices
  on or downstream of a directed cycle.
* Condensation levels respect every edge (Section 4.1, topological order).
* Tables 2 and 3 (Section 5.2): structural statistics of the controlled
  dependency regimes, exact where the paper prints counts.
* Theorem 1 (Section 4.2): every nontrivial SCC block has rho(W_CC) < 1 and a
  nonnegative inverse; hence q >= 0 gives dT >= 0.
* eq. (reversal): every traveltime-order-violating face satisfies the
  coordinate-wise reversal criterion.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from oracle import diag
from oracle.assembly import assemble_workload, face_coefficients


def _random_graph(rng, n, p):
    m = rng.uniform(size=(n, n)) < p
    np.fill_diagonal(m, False)
    j, i = np.nonzero(m)
    return j.astype(np.int64), i.astype(np.int64)


def _reach(n, j, i):
    R = np.eye(n, dtype=bool)
    R[j, i] = True
    for k in range(n):
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    return R


@pytest.mark.parametrize("seed", range(6))
def test_scc_matches_mutual_reachability(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 120))
    j, i = _random_graph(rng, n, 1.5 / n)
    W = sp.csr_matrix((np.full(j.shape[0], 0.5), (i, j)), shape=(n, n))
    _, lab = diag.scc_labels(W)
    R = _reach(n, j, i)
    mutual = R & R.T
    same = lab[:, None] == lab[None, :]
    assert np.array_equal(same, mutual)


@pytest.mark.parametrize("seed", range(6))
def test_kahn_residual_is_downstream_closure_of_cycles(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(30, 150))
    j, i = _random_graph(rng, n, 1.2 / n)
    R = _reach(n, j, i)
    on_cycle = np.zeros(n, dtype=bool)
    for a, b in zip(j, i):
        if R[b, a]:
            on_cycle[a] = on_cycle[b] = True
    expect = np.any(R[on_cycle], axis=0) if on_cycle.any() else np.zeros(n, dtype=bool)
    _, resolved = diag.kahn_levels(n, j, i)
    assert np.array_equal(~resolved, expect)


def test_condensation_levels_respect_edges():
    wl = W.curved_state(21, 21, 13, A=500.0, eps_T=0.05)
    op = assemble_workload(wl, 0)
    lab, clev, nlev = diag.condensation_levels(op.W)
    j, i = diag.edges(op.W)
    cross = lab[j] != lab[i]
    assert np.all(nlev[j][cross] < nlev[i][cross])
    assert np.all(nlev[j][~cross] == nlev[i][~cross])


def test_table2_regimes(golden):
    tab = golden("table2_regimes.json")
    for case in tab["cases"]:
        wl = W.curved_state(*tab["grid"], A=float(case["A_m"]), eps_T=float(case["eps_T_s"]))
        op = assemble_workload(wl, 0)
        fr = diag.fractions(op.W, wl.T[0])
        assert round(W.mu_g(wl.G, 3), 3) == pytest.approx(case["mu_G"], abs=1e-12)
        assert fr["n_scc"] == case["n_scc"]
        assert round(100 * fr["f_cyc"], 3) == pytest.approx(case["f_cyc_pct"], abs=1e-12)
        assert round(100 * fr["f_unr"], 3) == pytest.approx(case["f_unr_pct"], abs=1e-12)
        if case["largest_scc"] is not None:
            assert fr["largest_scc"] == case["largest_scc"]
        # f_vio differs from the printed value by a handful of edges out of
        # ~1.2e5 (counting convention not stated); approximate only
        assert 100 * fr["f_vio"] == pytest.approx(case["f_vio_pct"], abs=0.01)
        if case["case"] == "C":
            assert fr["n_cyc"] == tab["case_C_counts"]["n_cyc"]
            assert fr["n_unr"] == tab["case_C_counts"]["n_unr"]


@pytest.mark.slow
def test_table3_scc_refinement(golden):
    tab = golden("table3_scc_refinement.json")
    for row in tab["rows"]:
        wl = W.curved_state(*row["grid"], A=500.0, eps_T=0.05)
        op = assemble_workload(wl, 0)
        fr = diag.fractions(op.W, wl.T[0])
        assert fr["N"] == row["nodes"]
        assert fr["n_scc"] == row["n_scc"]
        assert fr["n_cyc"] == row["n_cyc"]
        assert fr["largest_scc"] == row["largest_scc"]
        assert fr["n_unr"] == row["n_unr"]
        assert round(fr["n_unr"] / fr["n_cyc"], 1) == pytest.approx(row["ratio"], abs=1e-9)


def test_theorem1_blocks_and_monotonicity():
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    op = assemble_workload(wl, 0)
    comps = diag.scc_summary(op.W)
    assert len(comps) == 6
    for comp in comps:
        rho = diag.block_spectral_radius(op.W, comp)
        assert rho < 1.0
        inv = diag.block_inverse(op.W, comp)
        assert np.all(inv >= -1e-14)
        # row sums inside the block are <= 1 and at least one is < 1
        Wcc = op.W[comp][:, comp].toarray()
        rs = Wcc.sum(axis=1)
        assert np.all(rs <= 1.0 + 1e-15) and np.any(rs < 1.0 - 1e-12)
    q = np.abs(np.random.default_rng(4).standard_normal(op.N))
    x = O.superlu_solve(op, q)
    assert np.all(x >= -1e-14 * np.abs(x).max())


def test_reversal_criterion_on_violating_faces():
    """eq. (reversal), written on the discrete face: an edge j -> i along axis d
    with T_j > T_i has T_d a^d < 0 on that face, i.e.
    g_d (sum_{d' != d} G_{d d'} g_{d'}) < -G_{dd} g_d^2."""
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    T = wl.T[0]
    op = assemble_workload(wl, 0)
    a_faces, g_faces = face_coefficients(3, wl.n1, wl.n2, wl.n3, wl.G, T)
    shape = (wl.n3, wl.n2, wl.n1)
    Gf = np.stack([wl.G[:, c] for c in range(6)], axis=1)
    full = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4,
            (1, 2): 5, (2, 1): 5}
    n_checked = 0
    for d in range(3):
        ax = 2 - d
        n = shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        ids = np.arange(wl.N).reshape(shape)
        plo, phi = ids[tuple(lo)], ids[tuple(hi)]
        a = a_faces[d]
        g = g_faces[d]
        Gface = {key: 0.5 * (Gf[:, full[key]].reshape(shape)[tuple(lo)]
                             + Gf[:, full[key]].reshape(shape)[tuple(hi)])
                 for key in [(d, 0), (d, 1), (d, 2)]}
        cross = sum(Gface[(d, dp)] * g[dp] for dp in range(3) if dp != d)
        diag_term = Gface[(d, d)] * g[d] ** 2
        # edges across this face and their direction
        fwd = (a > 0) & (op.W[phi.ravel(), plo.ravel()].A1.reshape(a.shape) > 0)
        bwd = (a < 0) & (op.W[plo.ravel(), phi.ravel()].A1.reshape(a.shape) > 0)
        vio = (fwd & (T[plo] > T[phi])) | (bwd & (T[phi] > T[plo]))
        lhs = g[d] * cross
        assert np.all(lhs[vio] < -diag_term[vio])
        n_checked += int(vio.sum())
    assert n_checked > 0


def _case_c_operator(T=None):
    from oracle.assembly import assemble
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    T = wl.T[0] if T is None else T
    return wl, assemble(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, T, wl.s, int(wl.src[0]))


def test_case_c_sccs_survive_traveltime_perturbation():
    """Section 5.2.2: small random perturbations of the stored traveltime
    leave case C's SCC structure (6 blocks, 82 cyclic nodes, Table 2)
    unchanged over a broad range - here every relative size from 1e-14 to
    1e-6, eight decades, for two seeds."""
    wl, op = _case_c_operator()
    base = diag.scc_summary(op.W)
    assert len(base) == 6 and sum(len(c) for c in base) == 82
    for seed in (0, 1):
        for eps in (1e-14, 1e-12, 1e-10, 1e-8, 1e-6):
            Tp = diag.perturbed_traveltime(wl.T[0], int(wl.src[0]), eps, seed)
            _, opp = _case_c_operator(Tp)
            assert diag.same_partition(diag.scc_summary(opp.W), base), (seed, eps)


def test_case_c_sccs_survive_weak_edge_cutoff():
    """Section 5.2.2: removing ever weaker-to-stronger dependencies does not
    eliminate all nontrivial SCCs until the cutoff is far above roundoff:
    cutoffs up to 1e-4 leave the partition unchanged, and the largest cutoff
    at which a cyclic block survives is above 1e-3 (it is 1.5e-2 here); just
    above it none is left."""
    wl, op = _case_c_operator()
    base = diag.scc_summary(op.W)
    for tau in (1e-15, 1e-12, 1e-9, 1e-6, 1e-4):
        assert diag.same_partition(diag.scc_summary(diag.weak_edge_cutoff(op.W, tau)), base), tau
    tau = diag.scc_survival_cutoff(op.W)
    assert tau > 1e-3
    assert diag.scc_summary(diag.weak_edge_cutoff(op.W, tau))
    assert not diag.scc_summary(diag.weak_edge_cutoff(op.W, np.nextafter(tau, 1.0)))


def test_survival_cutoff_closed_form():
    """On a hand-made graph the survival cutoff is the weakest edge of the
    strongest cycle: cycles 0->1->0 (weights 0.5, 0.2) and 2->3->4->2
    (weights 0.3, 0.4, 0.1) give max(min(0.5, 0.2), min(0.3, 0.4, 0.1)) = 0.2;
    an acyclic graph gives 0."""
    # W[i, j] = w_ij is the weight of edge j -> i
    ij = {(1, 0): 0.5, (0, 1): 0.2, (3, 2): 0.3, (4, 3): 0.4, (2, 4): 0.1, (4, 0): 0.9}
    W = sp.csr_matrix((list(ij.values()), ([i for i, _ in ij], [j for _, j in ij])), shape=(5, 5))
    assert diag.scc_survival_cutoff(W) == 0.2
    dag = sp.csr_matrix(([0.3, 0.7], ([1, 2], [0, 1])), shape=(3, 3))
    assert diag.scc_survival_cutoff(dag) == 0.0
