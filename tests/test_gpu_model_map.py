"""The cell-velocity model map M_alpha (Section 4.4, eq. (source-jacobian))
on the GPU, alone and around the transport.

* M dv and M^T g against the oracle's explicit derivative matrix: FP64 at
  1e-14 (sums of at most eight terms), FP32 at 1e-6; the adjoint pairing
  <M dv, g> = <dv, M^T g> at 1e-13;
* the background slowness the library derives from the cell velocities
  equals the oracle's; nonpositive velocities and too small grids are
  rejected;
* J M (M dv broadcast into fm_apply_J, receivers out) and M^T J^T (summed
  transpose, then M^T) against P A^-1 C M and M^T C A^-T P^T of the oracle at
  1e-11, with the pairing at 1e-12.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import oracle_ops, rel_l2, rel_l2_pairs, states_for
from oracle.model_map import cell_count, cell_slowness, model_map_matrix

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("g", [(3, 41, 37, 21), (2, 161, 1, 81)], ids=["3d", "2d"])
def test_map_and_transpose_against_oracle(g):
    dim, n1, n2, n3 = g
    print(f"case model map {g}", flush=True)
    Nc = cell_count(dim, n1, n2, n3)
    rng = np.random.default_rng(5100 + dim)
    v = rng.uniform(1.6, 3.2, Nc)
    Mo = model_map_matrix(dim, n1, n2, n3, v)
    N = Mo.shape[0]
    m = fm.ModelMap(dim, n1, n2, n3, v)
    assert (m.N, m.n_cells) == (N, Nc)
    assert np.allclose(m.slowness(), cell_slowness(dim, n1, n2, n3, v), rtol=1e-15, atol=0)
    B = 16
    dv = rng.standard_normal((Nc, B))
    gn = rng.standard_normal((N, B))
    for dt, tol in ((torch.float64, 1e-14), (torch.float32, 1e-6)):
        x = torch.from_numpy(dv).to("cuda", dt)
        y = torch.from_numpy(gn).to("cuda", dt)
        ds = torch.full((N, B), float("nan"), device="cuda", dtype=dt)
        mt = torch.full((Nc, B), float("nan"), device="cuda", dtype=dt)
        m.apply(x, ds)
        m.apply_T(y, mt)
        torch.cuda.synchronize()
        a, b = ds.double().cpu().numpy(), mt.double().cpu().numpy()
        assert rel_l2(a, Mo @ dv) <= tol and rel_l2(b, Mo.T @ gn) <= tol
        if dt == torch.float64:
            l, r = float(np.sum(a * gn)), float(np.sum(dv * b))
            assert abs(l - r) / max(abs(l), abs(r)) <= 1e-13
    m.free()
    bad = v.copy()
    bad[7] = -1.0
    with pytest.raises(fm.FmError):
        fm.ModelMap(dim, n1, n2, n3, bad)
    with pytest.raises(fm.FmError):
        fm.ModelMap(dim, 1, n2, n3, v)


def test_jacobian_with_cell_model():
    wl = W.grids.deformed_3d(41, 37, 21, 5200, 2, 2, 16, 6, 6, name="cells 41x37x21")
    v = W.cell_velocities(wl)
    m = fm.ModelMap(3, wl.n1, wl.n2, wl.n3, v)
    wl.s = m.slowness()
    W.eikonal(wl)
    states, ops = states_for(fm, wl), oracle_ops(wl)
    Mo = model_map_matrix(3, wl.n1, wl.n2, wl.n3, v)
    S, B, R, N, Nc = wl.S, 16, wl.rcv.shape[0], wl.N, m.n_cells
    print(f"case J M, S={S} B={B} R={R} cells={Nc}", flush=True)
    rng = np.random.default_rng(5201)
    dv = rng.standard_normal((Nc, B))
    y = rng.standard_normal((S, R, B))
    batch = fm.Batch(states, B, fm.FM_FP64)
    dev = torch.device("cuda")
    ds = torch.empty((N, B), device=dev, dtype=torch.float64)
    m.apply(torch.from_numpy(dv).to(dev), ds)
    d = torch.full((S, R, B), float("nan"), device=dev, dtype=torch.float64)
    batch.apply_J(ds, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
    g = torch.empty((N, B), device=dev, dtype=torch.float64)
    batch.apply_JT(torch.from_numpy(y).to(dev), fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
    gc = torch.full((Nc, B), float("nan"), device=dev, dtype=torch.float64)
    m.apply_T(g, gc)
    torch.cuda.synchronize()
    batch.status()
    jm = d.cpu().numpy()
    mtjt = gc.cpu().numpy()
    ds_o = Mo @ dv
    ref_j = np.stack([O.apply_J(op, ds_o, "receivers") for op in ops])
    assert rel_l2_pairs(jm, ref_j) <= 1e-11
    ref_t = Mo.T @ O.apply_JT_summed(ops, list(y), "receivers")
    assert rel_l2(mtjt, ref_t) <= 1e-11
    a, b = float(np.sum(jm * y)), float(np.sum(dv * mtjt))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-12
    batch.free()
    m.free()
