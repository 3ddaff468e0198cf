"""Benchmark: paired J + J^T applications per second over sources x right-hand
sides, the primal and transpose frozen full-metric tangent transport through
the SCC condensation graph (Algorithm 1, Phase III), on one MI355X.

One step = one LSQR iteration of the Krylov inner loop (Algorithm 1, Section 4.5)
over the whole batch: J from the model block [N][B] (broadcast to every
source) to receiver data [S][R][B], J^T back to the source-summed model block
(Section 4.4), and the LSQR vector updates.  The iterations run from a HIP
graph that records 30 of them and is replayed.  Inputs are resident in HBM
before the timed region.  Setup (Phase I) runs once before timing and is
reported separately.  The roofline figures use HIP events around eager
apply_J / apply_JT launches of the same batch on the same stream.

Prints one JSON line.  Default workload: the 201 x 201 x 101 deformed 3-D grid,
64 sources x 16 right-hand sides, 400 surface receivers, FP64.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(stats_list, B, vbytes, wbytes):
    """Compulsory HBM bytes of one launch of a sweep kernel, summed over
    sources: the input and output vectors once per (source, rhs)
    (2 * vbytes * N * B) plus the source's packed state read once - an 8-byte
    meta word and a 4-entry value record per node (8 + 4 * wbytes) and the FP64
    SCC block matrix of that direction (8 * sum k^2).  Predecessor re-reads
    and the records' overflow entries (<0.5 % of nodes) are not counted."""
    total = 0
    for st in stats_list:
        N, k2 = st["N"], st["sum_k2"]
        total += 2 * vbytes * N * B + (8 + 4 * wbytes) * N + 8 * k2
    return total


KERNEL_SOURCES = ("paper_2609_14982_amd/csrc/sweep.h", "paper_2609_14982_amd/csrc/split.h",
                  "paper_2609_14982_amd/csrc/device.hip", "paper_2609_14982_amd/csrc/setup.cpp")


def measured_traffic(kernel, config, precision):
    """HBM bytes per launch of the primal sweep kernel from the committed
    counter profile, or None when that profile is for another workload or for
    different kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{config}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    h = hashlib.sha256()
    for src in doc.get("kernel_sources", KERNEL_SOURCES):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != doc.get("kernel_source_sha256"):
        return None
    return doc["per_launch"]["J"]["hbm_bytes"]


def cpu_baseline(wl, n_src, B, seed):
    """The CPU oracle (explicit assembly + Gauss-Seidel directional sweeping to
    convergence, plain C, OpenMP over right-hand sides) on a bounded sample."""
    import oracle as O
    from oracle.assembly import assemble_workload

    threads = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((wl.N, B))
    y = rng.standard_normal((wl.rcv.shape[0], B))
    t0 = time.perf_counter()
    cycles = []
    for a in range(n_src):
        op = assemble_workload(wl, a)
        q = op.c[:, None] * p
        x, cy1 = O.gs_solve(op, op.W, q, nthreads=threads, return_cycles=True)
        r = O.solve.scatter_receivers(op, y)
        lam, cy2 = O.gs_solve(op, op.WT(), r, nthreads=threads, return_cycles=True)
        cycles += list(cy1) + list(cy2)
    dt = time.perf_counter() - t0
    pairs = n_src * B
    return {"value": pairs / dt, "unit": "paired applies/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_src} source(s) x {B} rhs of the same workload, J (broadcast p -> nodes) + "
                      f"J^T (receivers -> nodes), Gauss-Seidel sweeping to convergence "
                      f"(mean {np.mean(cycles):.1f} cycles of {2 ** wl.dim} sweeps), assembly included; "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="LSQR iterations timed (rounded up to 30s)")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default="c4", choices=["c2", "c3", "c4"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--sources", type=int, default=0, help="use only the first S sources (0: all)")
    ap.add_argument("--rhs-per-group", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--split", type=int, default=0, help="workgroups per source (0: library choice, 1: rhs groups)")
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--balance", type=int, default=0,
                    help="node split with workgroups per source from its level count (1-5: per-level weight)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the schedule search (fm_autotune) and use the library's choice or the flags")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sources", type=int, default=4)
    ap.add_argument("--no-sweep", action="store_true", help="skip the directional-sweeping comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of a known size (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = 1 << 29      # 2^29 doubles = 4 GiB read + 4 GiB written per copy
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                          "copies": 3}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2609_14982_amd as fm
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")

    t0 = time.perf_counter()
    wl = W.config(args.config, with_T=False)
    if args.sources:
        wl.src = wl.src[: args.sources]
    log(f"workload {args.config}: grid {wl.n1}x{wl.n2}x{wl.n3} N={wl.N} S={wl.S} B={wl.B} "
        f"R={wl.rcv.shape[0]} ({time.perf_counter() - t0:.1f}s)")
    t1 = time.perf_counter()
    W.eikonal(wl)
    log(f"first-arrival traveltimes for {wl.S} sources: {time.perf_counter() - t1:.1f}s")
    t1 = time.perf_counter()
    states = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src, wl.rcv)
    setup_wall = time.perf_counter() - t1
    stats = [st.stats() for st in states]
    log(f"setup (host, {min(16, os.cpu_count() or 1)} threads): {setup_wall:.1f}s; "
        f"levels fwd max {max(s['levels_fwd'] for s in stats)}, SCCs {sum(s['n_scc'] for s in stats)}, "
        f"largest {max(s['largest_scc'] for s in stats)}")

    prec = fm.FM_FP64 if args.precision == "fp64" else fm.FM_FP32
    dt = torch.float64 if prec == fm.FM_FP64 else torch.float32
    vbytes = 8 if prec == fm.FM_FP64 else 4
    tuning = {}
    if args.rhs_per_group:
        tuning["rhs_per_group"] = args.rhs_per_group
    if args.threads:
        tuning["threads"] = args.threads
    if args.split:
        tuning["split"] = args.split
    if args.unroll:
        tuning["unroll"] = args.unroll
    if args.balance:
        tuning["balance"] = args.balance
    S, N, B, R = wl.S, wl.N, wl.B, wl.rcv.shape[0]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    gen = torch.Generator(device=dev)
    gen.manual_seed(4000)
    p = torch.randn((N, B), device=dev, dtype=dt, generator=gen)
    y = torch.randn((S, R, B), device=dev, dtype=dt, generator=gen)
    d = torch.empty((S, R, B), device=dev, dtype=dt)
    g = torch.empty((N, B), device=dev, dtype=dt)
    tune_table = None
    if not args.no_autotune and not tuning:
        # schedule search on this batch's own data (outside the timed region)
        t1 = time.perf_counter()
        tuning, tune_table = fm.autotune(states, B, prec, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                                         y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED, reps=2, stream=stream)
        for t, ms in tune_table:
            log(f"autotune: split {t['split']} threads {t['threads']} unroll {t['unroll']} "
                f"balance {t.get('balance', 0)} rhs_per_group {t['rhs_per_group']}: {ms:.2f} ms per J + J^T")
        log(f"autotune: {time.perf_counter() - t1:.1f}s, best {tuning}")
    t1 = time.perf_counter()
    batch = fm.Batch(states, B, prec, tuning=tuning or None, stream=stream)
    torch.cuda.synchronize()
    log(f"batch create + upload: {time.perf_counter() - t1:.1f}s, tuning {batch.tuning()}")

    # the timed loop: LSQR iterations replayed from a captured graph
    GRAPH_ITERS = 30
    lsqr = fm.Lsqr(batch)
    lsqr.start(y)
    lsqr.capture(GRAPH_ITERS)
    n_warm = -(-args.warmup // GRAPH_ITERS)
    n_rep = max(1, -(-args.steps // GRAPH_ITERS))
    steps = n_rep * GRAPH_ITERS
    for _ in range(n_warm):
        lsqr.replay()
    torch.cuda.synchronize()
    log(f"warmup {n_warm * GRAPH_ITERS} LSQR iterations done")
    lsqr.start(y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream)
    for _ in range(n_rep):
        lsqr.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = max(wall * 1e3, ev0.elapsed_time(ev1)) / steps
    phibar = np.abs(lsqr.scalars().cpu().numpy()[3])
    log(f"timed {steps} LSQR iterations ({n_rep} graph replays): {ms_per_step:.3f} ms/iteration; "
        f"relative residual after {steps}: {np.median(phibar / np.linalg.norm(y.cpu().numpy().reshape(-1, B), axis=0)):.3e}")
    lsqr.free()

    # kernel durations for the roofline: events around eager applies
    def step(evs):
        evs[0].record(stream)
        batch.apply_J(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
        evs[1].record(stream)
        batch.apply_JT(y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
        evs[2].record(stream)

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(4)]
    for k in range(4):
        step(events[k])
    torch.cuda.synchronize()
    tJ = np.array([e[0].elapsed_time(e[1]) for e in events[1:]])
    tT = np.array([e[1].elapsed_time(e[2]) for e in events[1:]])
    log(f"eager applies: J {tJ.mean():.3f} ms, J^T {tT.mean():.3f} ms")

    # roofline of the dominant kernel: the primal sweep (one launch per apply_J,
    # between a counter reset of S words and the receiver gather of S*R*B
    # values, together <0.1 % of the window)
    split = batch.tuning()["split"] > 1
    kname = "k_split" if split else "k_sweep"
    bytes_J = algorithmic_bytes(stats, B, vbytes, vbytes)
    gbs_J = bytes_J / (tJ.mean() * 1e-3) / 1e9
    gbs_T = bytes_J / (tT.mean() * 1e-3) / 1e9
    traffic = measured_traffic(kname, args.config, args.precision) if not args.sources else None
    roof = {"bound": "hbm", "achieved": round(gbs_J, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs_J / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": f"{kname} primal (apply_J)", "bytes_per_launch": bytes_J,
            "launch_ms": round(float(tJ.mean()), 4),
            "transpose_GBs_incl_source_sum": round(gbs_T, 1)}
    # what a plain device copy sustains on this GPU (2 GiB read + 2 GiB
    # written per copy), and the primal kernel's counted bytes per second
    nc = 1 << 28
    ca = torch.ones(nc, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    cevs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    cb.copy_(ca)
    cevs[0].record(stream)
    for _ in range(5):
        cb.copy_(ca)
    cevs[1].record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nc * 8 * 5 / (cevs[0].elapsed_time(cevs[1]) * 1e-3) / 1e9
    del ca, cb
    roof["copy_GBs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(gbs_J / copy_gbs, 4)
    if traffic is not None:
        roof["traffic_GBs"] = round(traffic / (tJ.mean() * 1e-3) / 1e9, 1)
    log(f"device copy {copy_gbs:.0f} GB/s; primal kernel {gbs_J:.0f} GB/s algorithmic = {gbs_J / copy_gbs:.3f} of it")

    sweep = None
    if not args.no_sweep:
        # the same paired application by directional Gauss-Seidel sweeping
        # (Section 3.6) on the same GPU, converged to the same accuracy
        log("directional-sweeping comparison (converged)")
        rcv = torch.as_tensor(wl.rcv, device=dev)
        r_nodes = torch.zeros((S, N, B), device=dev, dtype=dt)
        batch.apply_J_sweep(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS, max_cycles=1)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        cj = batch.apply_J_sweep(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS, want_cycles=True)
        e1.record(stream)
        r_nodes.zero_()
        r_nodes.index_add_(1, rcv, y)      # P^T y at the nodes
        ct = batch.apply_JT_sweep(r_nodes, g, fm.FM_JT_SUMMED, want_cycles=True)
        e2.record(stream)
        torch.cuda.synchronize()
        tsJ, tsT = e0.elapsed_time(e1), e1.elapsed_time(e2)
        del r_nodes
        sweep = {"value": round(S * B / ((tsJ + tsT) * 1e-3), 3), "unit": "paired applies/s",
                 "J_ms": round(tsJ, 2), "JT_ms": round(tsT, 2),
                 "cycles_J": [int(cj.min()), int(cj.max())], "cycles_JT": [int(ct.min()), int(ct.max())],
                 "sweeps_per_cycle": 2 ** wl.dim}
        log(f"sweeping: J {tsJ:.1f} ms ({cj.min()}-{cj.max()} cycles), J^T {tsT:.1f} ms "
            f"({ct.min()}-{ct.max()} cycles)")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_sources} source(s) x {B} rhs")
        cpu = cpu_baseline(wl, args.cpu_sources, B, 4001)
        log(f"cpu baseline: {cpu['value']:.3f} paired applies/s")

    value = S * B / (ms_per_step * 1e-3)
    res = {
        "metric": "J+J^T paired applies/s (source x rhs) on a 3-D deformed grid, LSQR inner loop in a HIP graph",
        "value": round(value, 2),
        "unit": "paired applies/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": n_warm * GRAPH_ITERS,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fm.FM_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {wl.n1}x{wl.n2}x{wl.n3} deformed grid, "
                               f"{S} sources x {B} rhs, {R} receivers",
                   "schedule": batch.tuning(),
                   "schedule_search": ([{"split": t["split"], "threads": t["threads"], "unroll": t["unroll"],
                                         "balance": t.get("balance", 0), "min_lds_bytes": t["min_lds_bytes"],
                                         "ms": round(ms, 3)}
                                        for t, ms in tune_table] if tune_table else None),
                   "grid": [wl.n1, wl.n2, wl.n3], "sources": S, "rhs": B, "receivers": R,
                   "setup_s": round(setup_wall, 2),
                   "levels_fwd_max": max(s["levels_fwd"] for s in stats),
                   "n_scc_total": sum(s["n_scc"] for s in stats),
                   "largest_scc": max(s["largest_scc"] for s in stats),
                   "J_ms": round(float(tJ.mean()), 4), "JT_ms": round(float(tT.mean()), 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "vs_sweeping": round(value / sweep["value"], 2) if sweep else None,
        "sweeping_baseline": sweep,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
