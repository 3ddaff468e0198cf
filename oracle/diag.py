"""Graph diagnostics of the frozen transport (oracle; test infrastructure).

Section 3.3: edge j -> i iff w_ij > 0.
Section 3.4: traveltime-order violating edges (T_j > T_i), f_vio.
Section 3.5: Kahn elimination and its residual, f_unr (Proposition 2).
Section 4.1: strongly connected components and the condensation DAG.
Section 4.2: Theorem 1, rho(W_CC) < 1 and A_C^{-1} >= 0.
eq. (graph-fractions): f_vio = N_vio / N_E, f_cyc = N_cyc / N, f_unr = N_unr / N.

SCCs use scipy's strong-connectivity routine; it is pinned against brute-force
mutual reachability on small random digraphs (tests/test_oracle_graph.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def edges(W: sp.csr_matrix):
    """(j, i) arrays for every dependency edge j -> i (w_ij > 0)."""
    Wc = W.tocoo()
    m = Wc.data > 0.0
    return Wc.col[m].astype(np.int64), Wc.row[m].astype(np.int64)


def adjacency(W: sp.csr_matrix) -> sp.csr_matrix:
    """Adjacency with entry [j, i] = 1 for each edge j -> i."""
    j, i = edges(W)
    N = W.shape[0]
    return sp.csr_matrix((np.ones(j.shape[0]), (j, i)), shape=(N, N))


def scc_labels(W: sp.csr_matrix):
    n, lab = connected_components(adjacency(W), directed=True, connection="strong")
    return n, lab


def scc_summary(W: sp.csr_matrix):
    """Nontrivial SCCs (size > 1) as a list of sorted node arrays."""
    n, lab = scc_labels(W)
    counts = np.bincount(lab, minlength=n)
    big = np.nonzero(counts > 1)[0]
    order = np.argsort(lab, kind="stable")
    starts = np.concatenate([[0], np.cumsum(counts)])
    comps = [np.sort(order[starts[c]:starts[c + 1]]) for c in big]
    return comps


def kahn_levels(N: int, src_nodes: np.ndarray, dst_nodes: np.ndarray):
    """Kahn elimination on the digraph with edges src -> dst.

    Returns (level, resolved): level[v] = 1 + max level of its predecessors
    (0 for vertices without predecessors), defined for resolved vertices; -1
    for the residual R that never reaches zero unresolved in-degree.
    """
    indeg = np.bincount(dst_nodes, minlength=N).astype(np.int64)
    order = np.argsort(src_nodes, kind="stable")
    s_sorted = src_nodes[order]
    d_sorted = dst_nodes[order]
    ptr = np.searchsorted(s_sorted, np.arange(N + 1))
    level = np.full(N, -1, dtype=np.int64)
    frontier = np.nonzero(indeg == 0)[0]
    lev = 0
    while frontier.size:
        level[frontier] = lev
        # successors of the frontier
        starts, ends = ptr[frontier], ptr[frontier + 1]
        cnt = ends - starts
        if cnt.sum() == 0:
            break
        idx = np.repeat(starts, cnt) + (np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt))
        succ = d_sorted[idx]
        np.subtract.at(indeg, succ, 1)
        cand = np.unique(succ)
        frontier = cand[(indeg[cand] == 0) & (level[cand] < 0)]
        lev += 1
    return level, level >= 0


def condensation_levels(W: sp.csr_matrix):
    """Longest-path levels of the SCC condensation DAG (Section 4.1).

    Returns (comp_label [N], comp_level [ncomp], node_level [N]).
    """
    N = W.shape[0]
    ncomp, lab = scc_labels(W)
    j, i = edges(W)
    cj, ci = lab[j], lab[i]
    m = cj != ci
    pairs = np.unique(np.stack([cj[m], ci[m]], axis=1), axis=0) if m.any() else np.zeros((0, 2), np.int64)
    clev, ok = kahn_levels(ncomp, pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64))
    assert ok.all(), "condensation graph must be acyclic"
    return lab, clev, clev[lab]


def fractions(W: sp.csr_matrix, T: np.ndarray):
    """eq. (graph-fractions) plus SCC statistics."""
    N = W.shape[0]
    j, i = edges(W)
    E = j.shape[0]
    n_vio = int(np.count_nonzero(T[j] > T[i]))
    comps = scc_summary(W)
    n_cyc = int(sum(c.shape[0] for c in comps))
    _, resolved = kahn_levels(N, j, i)
    n_unr = int(N - np.count_nonzero(resolved))
    return {
        "N": N, "E": E, "n_vio": n_vio, "f_vio": n_vio / E if E else 0.0,
        "n_scc": len(comps), "n_cyc": n_cyc, "f_cyc": n_cyc / N,
        "largest_scc": max((c.shape[0] for c in comps), default=0),
        "n_unr": n_unr, "f_unr": n_unr / N,
    }


def block_spectral_radius(W: sp.csr_matrix, comp: np.ndarray) -> float:
    """rho(W_CC) for one SCC by dense eigenvalues (Theorem 1)."""
    Wcc = W[comp][:, comp].toarray()
    return float(np.max(np.abs(np.linalg.eigvals(Wcc))))


def block_inverse(W: sp.csr_matrix, comp: np.ndarray) -> np.ndarray:
    Wcc = W[comp][:, comp].toarray()
    return np.linalg.inv(np.eye(comp.shape[0]) - Wcc)


def downstream_closure(N: int, j: np.ndarray, i: np.ndarray, seeds: np.ndarray) -> np.ndarray:
    """Boolean mask of vertices reachable from the seed set (seeds included)."""
    adj = sp.csr_matrix((np.ones(j.shape[0]), (j, i)), shape=(N, N))
    mark = np.zeros(N, dtype=bool)
    mark[seeds] = True
    frontier = np.nonzero(mark)[0]
    while frontier.size:
        nxt = adj[frontier].indices
        nxt = nxt[~mark[nxt]]
        nxt = np.unique(nxt)
        mark[nxt] = True
        frontier = nxt
    return mark


# ---------------------------------------------------------------------------
# Robustness of the cyclic blocks (Section 5.2.2): the SCCs are a structural
# feature of the frozen full-metric transport, not an artefact of retained
# precision or negligible coefficients, if (a) small random perturbations of
# the stored traveltime leave the SCC partition unchanged over a broad range,
# and (b) removing progressively larger weak dependencies eliminates all
# nontrivial SCCs only at cutoffs far above roundoff-level weights.
# ---------------------------------------------------------------------------

def perturbed_traveltime(T: np.ndarray, src: int, eps: float, seed: int) -> np.ndarray:
    """T (1 + eps xi) with seeded standard normal xi; the source keeps T = 0."""
    xi = np.random.default_rng(seed).standard_normal(T.shape)
    Tp = T * (1.0 + eps * xi)
    Tp[src] = 0.0
    return Tp


def same_partition(a, b) -> bool:
    """Whether two lists of nontrivial SCCs (sorted node arrays) are the same sets."""
    if len(a) != len(b):
        return False
    ka = sorted(a, key=lambda c: int(c[0]))
    kb = sorted(b, key=lambda c: int(c[0]))
    return all(np.array_equal(x, y) for x, y in zip(ka, kb))


def weak_edge_cutoff(W: sp.csr_matrix, tau: float) -> sp.csr_matrix:
    """W with every dependency of weight below tau removed."""
    Wt = W.tocsr(copy=True)
    Wt.data[Wt.data < tau] = 0.0
    Wt.eliminate_zeros()
    return Wt


def scc_survival_cutoff(W: sp.csr_matrix) -> float:
    """The largest tau such that keeping only the dependencies of weight
    >= tau still leaves a nontrivial SCC (0 if W has none): every cutoff above
    it removes all cyclic blocks.  Raising the cutoff only removes edges, so
    the test is monotone: bisection over the distinct edge weights."""
    w = np.unique(W.tocsr().data)
    w = w[w > 0]
    if not scc_summary(W):
        return 0.0
    lo, hi = 0, w.size      # keeping weights >= w[lo] leaves an SCC; >= w[hi] (or nothing) leaves none
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if scc_summary(weak_edge_cutoff(W, w[mid])):
            lo = mid
        else:
            hi = mid
    return float(w[lo])
