"""The oracle's pins must catch plausible mistakes (no GPU).

Each case plants one mistake in a copy of an oracle step, on the CPU, and
checks that at least one pin that guards that step fails: the Table 1 digits
(Section 5.1), the scaling identity (Section 3.2) or the transpose pairing
(Section 4.4).
"""
import numpy as np
import pytest

import oracle as O
import oracle.assembly as OA
import oracle.solve as OS
import workloads as W
from oracle.assembly import assemble_workload


def _faces_mutant(kind):
    orig = OA.face_coefficients

    def faces(dim, n1, n2, n3, G, T):
        shape = OA._grid_shape(dim, n1, n2, n3)
        Tg = np.asarray(T, dtype=np.float64).reshape(shape)
        Gm = OA._metric_full(np.asarray(G, dtype=np.float64), dim, shape)
        nd = len(shape)
        D = [OA._central(Tg, nd - 1 - dd) for dd in range(dim)]
        a_faces, g_faces = [], []
        for d in range(dim):
            ax = nd - 1 - d
            n = shape[ax]
            lo = OA._sl(nd, ax, slice(0, n - 1))
            hi = OA._sl(nd, ax, slice(1, n))
            g = []
            for dp in range(dim):
                if dp == d:
                    g.append(Tg[hi] - Tg[lo])
                elif kind == "tangential_at_p_only":
                    g.append(D[dp][lo])
                else:
                    g.append(0.5 * (D[dp][lo] + D[dp][hi]))
            a = 0.0
            for dp in range(dim):
                if kind == "drop_cross_term" and dp != d:
                    continue
                if kind == "transposed_metric_index":
                    Gf = 0.5 * (Gm[dp][(d + 1) % dim][lo] + Gm[dp][(d + 1) % dim][hi]) if dp != d \
                        else 0.5 * (Gm[d][d][lo] + Gm[d][d][hi])
                elif kind == "metric_at_p_only":
                    Gf = Gm[d][dp][lo]
                else:
                    Gf = 0.5 * (Gm[d][dp][lo] + Gm[d][dp][hi])
                a = a + Gf * g[dp]
            if kind == "flipped_sign":
                a = -a
            a_faces.append(a)
            g_faces.append(g)
        return a_faces, g_faces
    return faces, orig


def _table1_e2(n=(21, 21, 11)):
    wl, ds, dT = W.manufactured(*n)
    op = assemble_workload(wl, 0)
    x = O.dense_solve(op, op.c * ds) if op.N <= 6000 else O.superlu_solve(op, op.c * ds)
    r, h = wl.meta["r"], wl.meta["h"]
    k, j, i = np.meshgrid(np.arange(wl.n3), np.arange(wl.n2), np.arange(wl.n1), indexing="ij")
    outer = ((i == 0) | (i == wl.n1 - 1) | (j == 0) | (j == wl.n2 - 1)
             | (k == 0) | (k == wl.n3 - 1)).reshape(-1)
    m = (~outer) & (r > 3.0 * h)
    m[wl.src[0]] = False
    return float(f"{np.linalg.norm((x - dT)[m]) / np.linalg.norm(dT[m]):.4e}")


def test_unmutated_baseline():
    assert _table1_e2() == 1.9062e-2


@pytest.mark.parametrize("kind", ["drop_cross_term", "flipped_sign", "tangential_at_p_only",
                                  "transposed_metric_index", "metric_at_p_only"])
def test_face_mutations_fail_table1(monkeypatch, kind):
    faces, _ = _faces_mutant(kind)
    monkeypatch.setattr(OA, "face_coefficients", faces)
    assert _table1_e2() != 1.9062e-2


def test_calibration_mutation_fails_scaling(monkeypatch):
    wl = W.config("c1")
    orig = OA.assemble

    def mutant(*a, **k):
        op = orig(*a, **k)
        op.c = op.c * op.s      # planted: c = l instead of c = l / s
        return op
    monkeypatch.setattr(OA, "assemble", mutant)
    op = OA.assemble(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[0], wl.s, int(wl.src[0]))
    x = O.apply_J(op, -wl.s, "nodes", "dense")
    assert np.linalg.norm(x + wl.T[0]) / np.linalg.norm(wl.T[0]) > 1e-6


def test_untransposed_adjoint_fails_pairing(monkeypatch):
    wl = W.config("c1")
    op = assemble_workload(wl, 0)
    rng = np.random.default_rng(5)
    ds = rng.standard_normal(op.N)
    w = rng.standard_normal(op.N)
    orig = OS._solve
    monkeypatch.setattr(OS, "_solve", lambda op_, q, transpose, solver: orig(op_, q, False, solver))
    a = np.dot(OS.apply_J(op, ds), w)
    b = np.dot(ds, OS.apply_JT(op, w))
    assert abs(a - b) / max(abs(a), abs(b)) > 1e-6


def test_overwriting_receiver_scatter_fails_pairing(monkeypatch):
    wl = W.config("c1")
    op = assemble_workload(wl, 0)
    op.rcv = np.concatenate([op.rcv, op.rcv[:5]])
    rng = np.random.default_rng(6)
    ds = rng.standard_normal(op.N)
    y = rng.standard_normal(op.rcv.shape[0])

    def bad_scatter(op_, y_):
        r = np.zeros((op_.N,) + y_.shape[1:])
        r[op_.rcv] = y_
        return r
    monkeypatch.setattr(OS, "scatter_receivers", bad_scatter)
    a = np.dot(OS.apply_J(op, ds, "receivers"), y)
    b = np.dot(ds, OS.apply_JT(op, y, "receivers"))
    assert abs(a - b) / max(abs(a), abs(b)) > 1e-6
