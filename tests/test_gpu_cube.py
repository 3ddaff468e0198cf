"""The 26-neighbour (cube) stencil on the GPU against the oracle's cube
assembly (oracle.assembly.cube_couplings), through the C ABI.

* Small fixtures (3 sources on a deformed 3-D grid, the curved-wavefront
  fixture with SCC blocks, c1 in 2-D): J per pair at every node and from a
  broadcast block at the receivers, J^T from nodes per source and from
  receiver data summed over sources, FP64 at 1e-11 against SuperLU solves of
  the explicit operator (FP32 at 1e-4), the transpose pairing at 1e-12, for
  the library's schedule, the rhs groups, a uniform node split and the
  balanced split; every FP64 schedule gives the same bits.
* c3 at full size (101 x 101 x 51, 8 sources x 16 rhs) with the cube
  stencil: J and per-source J^T on three sampled sources against the
  oracle's converged Gauss-Seidel sweeping, and the pairing over all sources.
* the benchmark's workload (201 x 201 x 101, 64 sources x 16 rhs) with the
  cube stencil at the balanced split: J to nodes and receivers and
  per-source J^T on four sampled sources against the oracle's sweeping, the
  pairing over all sources.
* The GPU setup pass and the sweeping baseline refuse cube-stencil states,
  and a batch cannot mix stencils.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import gpu_run, oracle_J, oracle_JT, oracle_ops, rel_l2, rel_l2_pairs, seeded_ds, states_for
from oracle.assembly import assemble_workload

torch = pytest.importorskip("torch")
fm = pytest.importorskip("paper_2609_14982_amd")

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4
TOL_ADJ = 1e-12


def _three_sources():
    wl = W.smooth_3d(25, 23, 13, topo_amp=0.2, with_T=False)
    wl.src = np.array([wl.node(3, 4, 0), wl.node(12, 11, 0), wl.node(21, 18, 0)], dtype=np.int64)
    W.eikonal(wl)
    return wl


def _curved():
    wl = W.curved_state(41, 41, 25, A=500.0, eps_T=0.05)
    wl.rcv = np.array([wl.node(i, j, 0) for j in range(0, 41, 4) for i in range(0, 41, 4)], dtype=np.int64)
    return wl


CASES = {"deformed3d_S3": _three_sources, "curved_scc": _curved, "c1": lambda: W.config("c1")}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    wl = CASES[request.param]()
    wl.stencil = 26
    print(f"case cube stencil {request.param}: {wl.n1}x{wl.n2}x{wl.n3}, S={wl.S}", flush=True)
    states = states_for(fm, wl)
    assert all(s.stats()["E"] > 0 for s in states)
    return request.param, wl, states, oracle_ops(wl)


def _pairing(d, y, p, g):
    a = float(np.sum(d * y))
    b = float(np.sum(p * g))
    return abs(a - b) / max(abs(a), abs(b))


TUNINGS = [None, {"split": 1}, {"split": 8, "threads": 256, "unroll": 3},
           {"balance": 3, "threads": 256, "unroll": 3}]


@pytest.mark.parametrize("tuning", TUNINGS, ids=["library", "rhs_groups", "split8", "balanced"])
def test_every_mode_fp64(case, tuning):
    name, wl, states, ops = case
    B, R = 16, wl.rcv.shape[0]
    b = fm.Batch(states, B, fm.FM_FP64, tuning=tuning)
    used = b.tuning()
    b.free()
    print(f"  {name} schedule {used}", flush=True)
    if tuning is None or tuning.get("split", 0) != 1:
        assert used["split"] > 1
    ds = seeded_ds(wl, B, 4100)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tuning)
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= TOL64
    p = seeded_ds(wl, B, 4101, per_pair=False)
    d = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS, tuning)
    assert rel_l2_pairs(d, oracle_J(ops, p, False, out="receivers")) <= TOL64
    w = np.random.default_rng(4102).standard_normal((wl.S, wl.N, B))
    g1 = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE, tuning)
    assert rel_l2_pairs(g1, oracle_JT(ops, w)) <= TOL64
    y = np.random.default_rng(4103).standard_normal((wl.S, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tuning)
    assert rel_l2(g, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL64
    for k in range(B):
        assert _pairing(d[..., k], y[..., k], p[:, k], g[:, k]) <= TOL_ADJ


def test_schedules_bit_identical_fp64(case):
    name, wl, states, _ = case
    B = 16
    ds = seeded_ds(wl, B, 4200)
    w = np.random.default_rng(4201).standard_normal((wl.S, wl.N, B))
    ref = None
    for t in TUNINGS:
        x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, t)
        g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_SUMMED, t)
        if ref is None:
            ref = (x, g)
        else:
            assert np.array_equal(x, ref[0]) and np.array_equal(g, ref[1]), t


@pytest.mark.parametrize("tuning", [None, {"split": 1}, {"split": 8, "threads": 256, "unroll": 4}],
                         ids=["library", "rhs_groups", "split8"])
def test_fp32(case, tuning):
    name, wl, states, ops = case
    B, R = 16, wl.rcv.shape[0]
    ds = seeded_ds(wl, B, 4300)
    x = gpu_run(fm, torch, states, B, fm.FM_FP32, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES, tuning)
    assert rel_l2_pairs(x, oracle_J(ops, ds, True)) <= TOL32
    y = np.random.default_rng(4301).standard_normal((wl.S, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP32, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tuning)
    assert rel_l2(g, O.apply_JT_summed(ops, list(y), "receivers")) <= TOL32


def test_refusals():
    dev = torch.device("cuda:0")
    wl = W.config("c1")
    with pytest.raises(fm.FmError) as e:
        _gpu_setup_cube(wl, dev)
    assert e.value.code == fm.binding.FM_EINVAL and "face" in str(e.value)
    face = states_for(fm, wl)
    wl.stencil = 26
    cube = states_for(fm, wl)
    with pytest.raises(fm.FmError) as e:
        fm.Batch([cube[0], face[0]], 8, fm.FM_FP64)
    assert e.value.code == fm.binding.FM_EINVAL and "stencil" in str(e.value)
    b = fm.Batch(cube, 8, fm.FM_FP64)
    ds = torch.zeros((1, wl.N, 8), dtype=torch.float64, device=dev)
    out = torch.zeros_like(ds)
    with pytest.raises(fm.FmError) as e:
        b.apply_J_sweep(ds, fm.FM_DS_PER_PAIR, out, fm.FM_OUT_NODES)
    assert e.value.code == fm.binding.FM_EINVAL and "face" in str(e.value)
    b.free()


def _gpu_setup_cube(wl, dev):
    import ctypes as C
    lib = fm.binding.load()
    G = np.ascontiguousarray(wl.G, dtype=np.float64)
    g = fm.binding._grid(wl.dim, wl.n1, wl.n2, wl.n3, G, 26)
    T = torch.from_numpy(np.ascontiguousarray(wl.T)).to(dev)
    s = np.ascontiguousarray(wl.s, dtype=np.float64)
    src = np.ascontiguousarray(wl.src, dtype=np.int64)
    outs = (C.c_void_p * wl.S)()
    fm.binding._check(lib.fm_build_frozen_states_gpu(C.byref(g), wl.S, C.c_void_p(T.data_ptr()), s.ctypes.data,
                                                     src.ctypes.data, None, None, 0, 1, 1,
                                                     C.c_void_p(torch.cuda.current_stream().cuda_stream), outs))


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_c3_full_size_cube():
    wl = W.config("c3")
    wl.stencil = 26
    S, B, R = wl.S, wl.B, wl.rcv.shape[0]
    print(f"case cube stencil c3 101x101x51, S={S}, B={B}: building", flush=True)
    states = states_for(fm, wl)
    print("  levels fwd " + str([s.stats()["levels_fwd"] for s in states]) +
          " blocks " + str([s.stats()["n_scc"] for s in states]), flush=True)
    b = fm.Batch(states, B, fm.FM_FP64)
    print(f"  schedule {b.tuning()}", flush=True)
    assert b.tuning()["split"] > 1
    b.free()
    ds = seeded_ds(wl, B, 4400)
    x = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_NODES)
    w = np.random.default_rng(4401).standard_normal((S, wl.N, B))
    gps = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", w, fm.FM_W_NODES, fm.FM_JT_PER_SOURCE)
    threads = min(16, os.cpu_count() or 1)
    for a in (0, S // 2, S - 1):
        op = assemble_workload(wl, a)
        xo = O.gs_solve(op, op.W, op.c[:, None] * ds[a], nthreads=threads)
        ej = rel_l2_pairs(x[a:a + 1], xo[None])
        lam = O.gs_solve(op, op.WT(), w[a], nthreads=threads)
        et = rel_l2_pairs(gps[a:a + 1], (op.c[:, None] * lam)[None])
        print(f"  source {a}: J {ej:.2e}, J^T {et:.2e}", flush=True)
        assert ej <= TOL64 and et <= TOL64
    p = seeded_ds(wl, B, 4402, per_pair=False)
    d = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", p, fm.FM_DS_BROADCAST, fm.FM_OUT_RECEIVERS)
    y = np.random.default_rng(4403).standard_normal((S, R, B))
    g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED)
    for k in range(B):
        assert _pairing(d[..., k], y[..., k], p[:, k], g[:, k]) <= TOL_ADJ


def test_point_sources_with_cube_stencil():
    """Off-grid point sources (seed rows, the direct term D) on cube-stencil
    states: J to receivers and the summed J^T from receiver data against
    the point-source oracle with the cube stencil, FP64 at 1e-11, node split
    and rhs groups."""
    from oracle import source as PS
    wl = W.smooth_3d(21, 19, 11, topo_amp=0.15, with_T=False)
    xi = np.array([[6.3, 7.1, 0.0], [13.6, 11.2, 2.5], [3.0, 15.0, 0.0]])
    W.eikonal_point(wl, xi, 1.5)
    print("case cube stencil, point sources 21x19x11, S=3", flush=True)
    states = fm.build_frozen_states_pt(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, wl.T, wl.s, xi, 1.5, wl.rcv, stencil=26)
    psos = [PS.assemble_point_source(3, wl.n1, wl.n2, wl.n3, wl.G, wl.X, wl.T[a], wl.s, xi[a], 1.5, wl.rcv,
                                     stencil=26) for a in range(3)]
    B, R = 16, wl.rcv.shape[0]
    rng = np.random.default_rng(4500)
    ds = rng.standard_normal((3, wl.N, B))
    y = rng.standard_normal((3, R, B))
    ref_d = np.stack([PS.apply_J(psos[a], ds[a]) for a in range(3)])
    ref_g = sum(PS.apply_JT(psos[a], y[a]) for a in range(3))
    for tuning in (None, {"split": 1}):
        d = gpu_run(fm, torch, states, B, fm.FM_FP64, "J", ds, fm.FM_DS_PER_PAIR, fm.FM_OUT_RECEIVERS, tuning)
        g = gpu_run(fm, torch, states, B, fm.FM_FP64, "JT", y, fm.FM_W_RECEIVERS, fm.FM_JT_SUMMED, tuning)
        ed, eg = rel_l2_pairs(d, ref_d), rel_l2(g, ref_g)
        print(f"  {tuning}: J {ed:.2e}, J^T {eg:.2e}", flush=True)
        assert ed <= TOL64 and eg <= TOL64


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_c4_full_size_cube():
    """The benchmark's workload (201 x 201 x 101, 64 sources x 16 rhs, 400
    receivers) with the cube stencil, all 64 states in one batch at the
    balanced split with 256-thread workgroups: J from a broadcast block to
    every node and to the receivers, and per-source J^T from receiver data,
    on sampled sources (fewest and most block entries, deepest and shallowest
    forward schedules, the middle and the last source) against the oracle's
    converged Gauss-Seidel sweeping at 1e-11;
    the transpose pairing over all sources."""
    wl = W.config("c4")
    wl.stencil = 26
    S, B, R, N = wl.S, wl.B, wl.rcv.shape[0], wl.N
    print(f"case cube stencil c4 201x201x101, S={S}, B={B}: building", flush=True)
    states = states_for(fm, wl)
    st = [s.stats() for s in states]
    k2 = np.array([s["sum_k2"] for s in st])
    lf = np.array([s["levels_fwd"] for s in st])
    sample = sorted({int(np.argmin(k2)), int(np.argmax(k2)), int(np.argmax(lf)), int(np.argmin(lf)), S // 2, S - 1})
    print(f"  sampled sources {sample}: sum k^2 {k2[sample].tolist()}, levels fwd {lf[sample].tolist()}", flush=True)
    rng = np.random.default_rng(4600)
    p = W.smooth_noise(wl, B, rng)
    y = rng.standard_normal((S, R, B))
    dev = torch.device("cuda:0")
    batch = fm.Batch(states, B, fm.FM_FP64, tuning={"balance": 3, "threads": 256, "unroll": 3})
    used = batch.tuning()
    print(f"  schedule {used}", flush=True)
    assert used["split"] > 1
    d_p = torch.from_numpy(p).to(dev)
    d_y = torch.from_numpy(y).to(dev)
    idx = torch.tensor(sample, device=dev)
    big = torch.empty((S, N, B), dtype=torch.float64, device=dev)
    batch.apply_J(d_p, fm.FM_DS_BROADCAST, big, fm.FM_OUT_NODES)
    batch.status()
    xn = big.index_select(0, idx).cpu().numpy()
    d = torch.empty((S, R, B), dtype=torch.float64, device=dev)
    batch.apply_J(d_p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
    batch.apply_JT(d_y, fm.FM_W_RECEIVERS, big, fm.FM_JT_PER_SOURCE)
    g = torch.empty((N, B), dtype=torch.float64, device=dev)
    batch.apply_JT(d_y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
    batch.status()
    gn = big.index_select(0, idx).cpu().numpy()
    d, g = d.cpu().numpy(), g.cpu().numpy()
    del big
    batch.free()
    torch.cuda.empty_cache()
    threads = min(16, os.cpu_count() or 1)
    for i, a in enumerate(sample):
        op = assemble_workload(wl, a)
        xo = O.gs_solve(op, op.W, op.c[:, None] * p, nthreads=threads)
        r = O.solve.scatter_receivers(op, y[a])
        lam = O.gs_solve(op, op.WT(), r, nthreads=threads)
        e = (rel_l2_pairs(xn[i:i + 1], xo[None]), rel_l2_pairs(d[a:a + 1], xo[wl.rcv][None]),
             rel_l2_pairs(gn[i:i + 1], (op.c[:, None] * lam)[None]))
        print(f"  source {a}: J nodes {e[0]:.2e}, J receivers {e[1]:.2e}, J^T {e[2]:.2e}", flush=True)
        assert max(e) <= TOL64
    for k in range(B):
        assert _pairing(d[..., k], y[..., k], p[:, k], g[:, k]) <= TOL_ADJ
