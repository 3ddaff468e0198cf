"""Benchmark: paired J + J^T applications per second over sources x right-hand
sides, the primal and transpose frozen full-metric tangent transport through
the SCC condensation graph (Algorithm 1, Phase III), on one MI355X.

One step = one LSQR iteration of the Krylov inner loop (Algorithm 1, Section 4.5)
over the whole batch: J from the model block [N][B] (broadcast to every
source) to receiver data [S][R][B], J^T back to the source-summed model block
(Section 4.4), and the LSQR vector updates.  One iteration is captured as a
HIP graph; --warmup replays run untimed, then exactly --steps replays are
timed between two device synchronisations, with HIP events around every
replay for the median and spread.  Inputs are resident in HBM before the timed
region.  Setup (Phase I) runs once before timing and is reported separately.
The roofline figures use HIP events around 20 eager apply_J / apply_JT
launches of the same batch on the same stream.

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
    """Algorithmic bytes of one launch of a sweep kernel, summed over sources:
    per (source, rhs) the input and output vectors once (2 * vbytes * N), per
    source its state read once - per node the mean edge count times a weight
    and a 4-byte index, a calibration weight and two 4-byte indices
    (N * (ebar * (wbytes + 4) + 4 + wbytes + 4)) - and the FP64 SCC block
    matrix of that direction (8 * sum k^2 over the blocks kept as dense
    inverses; a block solved by its Neumann series reads its in-block
    couplings, a weight and a 4-byte index each, 12 * couplings).
    Predecessor re-reads and the series' re-reads of the couplings count as
    cache hits.  A broadcast input counts once per (source, rhs), as every
    source reads it."""
    total = 0
    for st in stats_list:
        N = st["N"]
        ebar = st["E"] / N
        blocks = 8 * st.get("dense_k2", st["sum_k2"]) + 12 * st.get("iter_nnz", 0)
        total += 2 * vbytes * N * B + N * (ebar * (wbytes + 4) + 4 + wbytes + 4) + blocks
    return int(round(total))


def layout_bytes(stats_list, B, vbytes, wbytes, broadcast_once=False):
    """Bytes the kernels move by design: input and output rows per (source,
    rhs), an 8-byte meta word and a 4-entry value record per node, the block
    matrix; with broadcast_once the shared input block is counted once."""
    total = 0
    for i, st in enumerate(stats_list):
        N, k2 = st["N"], st["sum_k2"]
        nin = 0 if (broadcast_once and i > 0) else 1
        total += (nin + 1) * vbytes * N * B + (8 + 4 * wbytes) * N + 8 * st.get("dense_k2", k2) + \
            12 * st.get("iter_nnz", 0)
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


def _csv_rows(root, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def _per_dispatch(root, counter):
    """{kernel name: [value per dispatch]} from a rocprofv3 --pmc run."""
    per = {}
    for r in _csv_rows(root, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id")))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def write_traffic(root, config, precision):
    """Fabric bytes per launch of the sweep kernels from four rocprofv3 --pmc
    runs (FETCH_SIZE and WRITE_SIZE of the benchmark and of a plain device
    copy of known size, KiB per dispatch), scaled so that the copy reads and
    writes what it moves; plus the trace's average durations."""
    import hashlib
    fetch = _per_dispatch(os.path.join(root, "fetch"), "FETCH_SIZE")
    write = _per_dispatch(os.path.join(root, "write"), "WRITE_SIZE")
    cf = _per_dispatch(os.path.join(root, "cfetch"), "FETCH_SIZE")
    cw = _per_dispatch(os.path.join(root, "cwrite"), "WRITE_SIZE")
    copy_bytes = (1 << 29) * 8
    ck = max(cf, key=lambda k: np.mean(cf[k]))
    cfk, cwk = float(np.mean(cf[ck])), float(np.mean(cw[max(cw, key=lambda k: np.mean(cw[k]))]))
    fscale, wscale = copy_bytes / (cfk * 1024), copy_bytes / (cwk * 1024)

    def pick(table, pattern):
        names = [k for k in table if pattern in k]
        if not names:
            return None, []
        name = max(names, key=lambda k: len(table[k]))
        return name, table[name]

    vt = "double" if precision == "fp64" else "float"
    per_launch = {}
    for label, pattern in (("J", f"k_split<0, {vt}"), ("JT", f"k_split<1, {vt}"), ("source_sum", f"k_sum_sources<{vt}")):
        name, fv = pick(fetch, pattern)
        _, wv = pick(write, pattern)
        if name is None or not wv:
            continue
        fk, wk = float(np.mean(fv)), float(np.mean(wv))
        per_launch[label] = {"kernel": name, "dispatches": len(fv), "fetch_kib": fk, "write_kib": wk,
                             "hbm_bytes": int(round(fk * 1024 * fscale + wk * 1024 * wscale))}
    stats = {}
    for r in _csv_rows(os.path.join(root, "trace"), "kernel_stats.csv"):
        if "k_split" in r["Name"] or "k_sum_sources" in r["Name"]:
            stats[r["Name"]] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"])}
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    doc = {"workload": f"{config}: {precision}, the benchmark's default batch", "kernel_sources": list(KERNEL_SOURCES),
           "kernel_source_sha256": h.hexdigest(),
           "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes, "copy_kernel": ck,
                                "fetch_kib_per_dispatch": cfk, "write_kib_per_dispatch": cwk,
                                "fetch_scale": fscale, "write_scale": wscale},
           "per_launch": per_launch, "kernel_stats_ns": stats}
    path = os.path.join(ROOT, "profiles", f"traffic_k_split_{config}_{precision}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({"written": path, "per_launch": per_launch}))


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


def level_histogram(states, stats):
    """Per source: levels, barriers per direction (one per level, one more
    per level holding SCC blocks), and the level-size distribution of the
    primal walk (nodes per level, deciles)."""
    out = []
    for a, (st, sd) in enumerate(zip(states, stats)):
        comp, lf, lr = st.export_graph()
        sizes = np.bincount(lf)
        szr = np.bincount(lr)
        # a level holds blocks when one of its components has more than one member
        ncomp = np.bincount(comp)
        big = ncomp[comp] > 1
        blk_f = np.unique(lf[big]).size
        blk_r = np.unique(lr[big]).size
        q = np.percentile(sizes, [0, 10, 25, 50, 75, 90, 100]).round(1).tolist()
        out.append({"source": a, "levels_fwd": int(sd["levels_fwd"]), "levels_rev": int(sd["levels_rev"]),
                    "barriers_fwd": int(sizes.size + blk_f), "barriers_rev": int(szr.size + blk_r),
                    "fwd_levels_lt_64_nodes": int(np.sum(sizes < 64)),
                    "fwd_levels_lt_256_nodes": int(np.sum(sizes < 256)),
                    "fwd_levels_lt_1024_nodes": int(np.sum(sizes < 1024)),
                    "fwd_nodes_in_levels_lt_256": int(sizes[sizes < 256].sum()),
                    "fwd_level_size_pctl_0_10_25_50_75_90_100": q, "n_scc": int(sd["n_scc"]),
                    "largest_scc": int(sd["largest_scc"]), "sum_k2": int(sd["sum_k2"])})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="LSQR iterations timed")
    ap.add_argument("--warmup", type=int, default=5, help="untimed LSQR iterations before the timed ones")
    ap.add_argument("--config", default="c4", choices=["c2", "c3", "c4"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--stencil", type=int, default=6, choices=[6, 26],
                    help="dependency stencil: 6 (face-based upwinding) or 26 (the cube variant)")
    ap.add_argument("--sources", type=int, default=0, help="use only the first S sources (0: all)")
    ap.add_argument("--rhs-per-group", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--split", type=int, default=0, help="workgroups per source (0: library choice, 1: rhs groups)")
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--balance", type=int, default=0,
                    help="node split with workgroups per source from a cost model (1-10, see fm_tuning)")
    ap.add_argument("--min-lds", type=int, default=0, help="LDS reserved per workgroup (limits occupancy)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the schedule search (fm_autotune) and use the library's choice or the flags")
    ap.add_argument("--no-tune-cache", action="store_true", help="search even when a cached schedule exists")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sources", type=int, default=4)
    ap.add_argument("--no-sweep", action="store_true", help="skip the directional-sweeping comparison")
    ap.add_argument("--no-gpu-setup", action="store_true",
                    help="skip timing the GPU setup pass on the same traveltimes (outside the timed region)")
    ap.add_argument("--roofline-reps", type=int, default=20, help="eager J and J^T launches timed for the roofline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of a known size (HBM counter calibration)")
    ap.add_argument("--level-histogram", action="store_true",
                    help="only build the states and print the level structure per source (no GPU)")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="only read the rocprofv3 outputs under DIR (fetch/, write/, cfetch/, cwrite/, trace/) "
                         "and write profiles/traffic_k_split_<config>_<precision>.json (no GPU)")
    args = ap.parse_args()

    tag = args.config + ("_cube" if args.stencil == 26 else "")
    if args.write_traffic:
        write_traffic(args.write_traffic, tag, args.precision)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; the path has no multi-GPU mode "
                                   "(--gpus must be 1)", "n_gpus": args.gpus}))
        sys.exit(2)

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

    import torch  # before the library, so that both use one HIP runtime

    import paper_2609_14982_amd as fm
    import workloads as W

    t0 = time.perf_counter()
    wl = W.config(args.config, with_T=False)
    wl.stencil = args.stencil
    if args.stencil == 26:
        args.no_sweep = True     # the sweeping baseline takes face-stencil states only
    if args.sources:
        wl.src = wl.src[: args.sources]
    log(f"workload {args.config}: grid {wl.n1}x{wl.n2}x{wl.n3} N={wl.N} S={wl.S} B={wl.B} "
        f"R={wl.rcv.shape[0]} ({time.perf_counter() - t0:.1f}s)")
    t1 = time.perf_counter()
    W.eikonal(wl)
    log(f"first-arrival traveltimes for {wl.S} sources: {time.perf_counter() - t1:.1f}s")
    t1 = time.perf_counter()
    states = fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T, wl.s, wl.src, wl.rcv,
                                    stencil=args.stencil)
    setup_wall = time.perf_counter() - t1
    stats = [st.stats() for st in states]
    log(f"setup (host, {min(16, os.cpu_count() or 1)} threads): {setup_wall:.1f}s; "
        f"levels fwd max {max(s['levels_fwd'] for s in stats)}, SCCs {sum(s['n_scc'] for s in stats)}, "
        f"largest {max(s['largest_scc'] for s in stats)}")
    if args.level_histogram:
        print(json.dumps({"workload": args.config, "grid": [wl.n1, wl.n2, wl.n3], "N": wl.N,
                          "per_source": level_histogram(states, stats)}), flush=True)
        return

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")

    setup_gpu = None
    if args.stencil == 6 and not args.no_gpu_setup:
        # the same states from the GPU setup pass, timed for the record (the
        # applies below use the host-built states; the two give the same bits)
        Td = torch.from_numpy(np.ascontiguousarray(wl.T)).to(dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gstates = fm.build_frozen_states_gpu(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, Td, wl.s, wl.src, wl.rcv)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t1
        keys = ("N", "E", "n_scc", "largest_scc", "levels_fwd", "levels_rev", "sum_k2")
        same = all(g.stats()[k] == h[k] for g, h in zip(gstates, stats) for k in keys)
        for gs in gstates:
            gs.free()
        del gstates, Td
        setup_gpu = {"seconds": round(tg, 2), "same_structure_as_host": bool(same)}
        log(f"setup (GPU pass, same traveltimes): {tg:.2f}s; structure {'matches' if same else 'DIFFERS from'} the host's")

    prec = fm.FM_FP64 if args.precision == "fp64" else fm.FM_FP32
    dt = torch.float64 if prec == fm.FM_FP64 else torch.float32
    vbytes = 8 if prec == fm.FM_FP64 else 4
    tuning = {}
    for k, v in (("rhs_per_group", args.rhs_per_group), ("threads", args.threads), ("split", args.split),
                 ("unroll", args.unroll), ("balance", args.balance), ("min_lds_bytes", args.min_lds)):
        if v:
            tuning[k] = v
    S, N, B, R = wl.S, wl.N, wl.B, wl.rcv.shape[0]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    gen = torch.Generator(device=dev)
    gen.manual_seed(4000)
    p = torch.randn((N, B), device=dev, dtype=dt, generator=gen)
    y = torch.randn((S, R, B), device=dev, dtype=dt, generator=gen)
    d = torch.empty((S, R, B), device=dev, dtype=dt)
    g = torch.empty((N, B), device=dev, dtype=dt)
    tune_table, tune_cached = None, False
    if not args.no_autotune and not tuning:
        # schedule search on this batch's own data (outside the timed region),
        # or the schedule an earlier search stored for the same device, batch
        # and state structure
        t1 = time.perf_counter()
        tuning, tune_table = fm.autotune(states, B, prec, p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS,
                                         y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED, reps=2, stream=stream,
                                         cache=not args.no_tune_cache)
        tune_cached = not tune_table
        for t, ms in tune_table:
            log(f"autotune: split {t['split']} threads {t['threads']} unroll {t['unroll']} "
                f"balance {t.get('balance', 0)} rhs_per_group {t['rhs_per_group']}: {ms:.2f} ms per J + J^T")
        log(f"autotune: {time.perf_counter() - t1:.1f}s, best {tuning}{' (cached)' if tune_cached else ''}")
    t1 = time.perf_counter()
    batch = fm.Batch(states, B, prec, tuning=tuning or None, stream=stream)
    torch.cuda.synchronize()
    log(f"batch create + upload: {time.perf_counter() - t1:.1f}s, tuning {batch.tuning()}")

    # the timed loop: LSQR iterations, each one replay of a captured graph
    lsqr = fm.Lsqr(batch)
    lsqr.start(y)
    lsqr.capture(1)
    for _ in range(args.warmup):
        lsqr.replay()
    torch.cuda.synchronize()
    batch.status()
    log(f"warmup {args.warmup} LSQR iterations done")
    lsqr.start(y)
    steps = max(1, args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    evs[0].record(stream)
    for k in range(steps):
        lsqr.replay()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    batch.status()
    per_it = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    ms_per_step = max(wall * 1e3, evs[0].elapsed_time(evs[-1])) / steps
    phibar = np.abs(lsqr.scalars().cpu().numpy()[3])
    log(f"timed {steps} LSQR iterations: {ms_per_step:.3f} ms/iteration (median {np.median(per_it):.3f}, "
        f"min {per_it.min():.3f}, max {per_it.max():.3f}); relative residual after {steps}: "
        f"{np.median(phibar / np.linalg.norm(y.cpu().numpy().reshape(-1, B), axis=0)):.3e}")
    lsqr.free()

    # kernel durations for the roofline: events around eager applies
    reps = max(1, args.roofline_reps)
    eJ = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps + 1)]
    eT = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps + 1)]
    for k in range(reps + 1):
        eJ[k][0].record(stream)
        batch.apply_J(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
        eJ[k][1].record(stream)
    for k in range(reps + 1):
        eT[k][0].record(stream)
        batch.apply_JT(y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
        eT[k][1].record(stream)
    torch.cuda.synchronize()
    batch.status()
    tJ = np.array([e[0].elapsed_time(e[1]) for e in eJ[1:]])
    tT = np.array([e[0].elapsed_time(e[1]) for e in eT[1:]])
    log(f"eager applies ({reps} each): J {tJ.mean():.3f} ms (median {np.median(tJ):.3f}), "
        f"J^T {tT.mean():.3f} ms (median {np.median(tT):.3f})")
    # the node split's placement in the last launch: sources whose workgroups
    # all ran on one XCD exchange their node values through one L2 (the
    # others paid device-scope fences at every level)
    placement = None
    if batch.tuning()["split"] > 1:
        xm = batch.split_info()
        one = int(sum(1 for m in xm if bin(int(m) & 0xFFFFFFFF).count("1") == 1))
        placement = {"sources_on_one_xcd": one, "sources": int(len(xm))}
        log(f"node split placement: {one} of {len(xm)} sources on one XCD")

    # roofline of the dominant kernel: the primal sweep (one launch per apply_J,
    # between a counter reset of S words and the receiver gather of S*R*B
    # values, together <0.1 % of the window)
    split = batch.tuning()["split"] > 1
    kname = "k_split" if split else "k_sweep"
    bytes_J = algorithmic_bytes(stats, B, vbytes, vbytes)
    gbs_J = bytes_J / (tJ.mean() * 1e-3) / 1e9
    gbs_T = bytes_J / (tT.mean() * 1e-3) / 1e9
    traffic = measured_traffic(kname, tag, args.precision) if not args.sources else None
    roof = {"bound": "hbm", "achieved": round(gbs_J, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs_J / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_kind": "fabric bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a plain copy "
                            "of known size; they include reads served by the memory-side cache",
            "kernel": f"{kname} primal (apply_J)",
            "bytes_per_launch": bytes_J,
            "bytes_model": "per (source, rhs) 2*vbytes*N, per source N*(ebar*(wbytes+4)+4+wbytes+4) + 8*sum k^2",
            "bytes_layout": layout_bytes(stats, B, vbytes, vbytes),
            "bytes_layout_broadcast_once": layout_bytes(stats, B, vbytes, vbytes, broadcast_once=True),
            "launch_ms": round(float(tJ.mean()), 4), "launch_ms_median": round(float(np.median(tJ)), 4),
            "launches_timed": reps,
            "placement": placement,
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
        roof["traffic_over_algorithmic"] = round(traffic / bytes_J, 3)
    log(f"device copy {copy_gbs:.0f} GB/s; primal kernel {gbs_J:.0f} GB/s algorithmic = {gbs_J / PEAK_HBM_GBS:.3f} "
        f"of peak, {gbs_J / copy_gbs:.3f} of the copy")

    sweep = None
    if not args.no_sweep:
        # the same paired application by directional Gauss-Seidel sweeping
        # (Section 3.6) on the same GPU, converged, checked against the
        # SCC/BTF outputs before its rate is reported
        log("directional-sweeping comparison (converged)")
        batch.apply_J(p, fm.FM_DS_BROADCAST, d, fm.FM_OUT_RECEIVERS)
        batch.apply_JT(y, fm.FM_W_RECEIVERS, g, fm.FM_JT_SUMMED)
        batch.status()
        d_ref, g_ref = d.clone(), g.clone()
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

        def rel_pairs(x, ref):
            """max over (source, rhs) of the relative l2 difference; [S][*][B] or [*][B]"""
            x, ref = x.double(), ref.double()
            if x.dim() == 2:
                x, ref = x[None], ref[None]
            num = torch.linalg.vector_norm(x - ref, dim=-2)
            den = torch.linalg.vector_norm(ref, dim=-2).clamp_min(1e-300)
            return float((num / den).max())
        errJ, errT = rel_pairs(d, d_ref), rel_pairs(g, g_ref)
        tol = 1e-11 if prec == fm.FM_FP64 else 1e-4
        sweep = {"value": round(S * B / ((tsJ + tsT) * 1e-3), 3), "unit": "paired applies/s",
                 "J_ms": round(tsJ, 2), "JT_ms": round(tsT, 2),
                 "cycles_J": [int(cj.min()), int(cj.max())], "cycles_JT": [int(ct.min()), int(ct.max())],
                 "sweeps_per_cycle": 2 ** wl.dim,
                 "rel_l2_vs_scc_btf_J": errJ, "rel_l2_vs_scc_btf_JT": errT, "agreement_tol": tol,
                 "agrees": bool(errJ <= tol and errT <= tol)}
        log(f"sweeping: J {tsJ:.1f} ms ({cj.min()}-{cj.max()} cycles), J^T {tsT:.1f} ms "
            f"({ct.min()}-{ct.max()} cycles); max rel l2 against SCC/BTF: J {errJ:.2e}, J^T {errT:.2e}")

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
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_median": round(float(np.median(per_it)), 4),
        "ms_per_step_min_max": [round(float(per_it.min()), 4), round(float(per_it.max()), 4)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fm.FM_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {wl.n1}x{wl.n2}x{wl.n3} deformed grid, "
                               f"{S} sources x {B} rhs, {R} receivers"
                               + (", 26-neighbour cube stencil" if args.stencil == 26 else ""),
                   "stencil": args.stencil,
                   "schedule": batch.tuning(),
                   "schedule_cached": tune_cached,
                   "schedule_search": ([{"split": t["split"], "threads": t["threads"], "unroll": t["unroll"],
                                         "balance": t.get("balance", 0), "min_lds_bytes": t["min_lds_bytes"],
                                         "ms": round(ms, 3)}
                                        for t, ms in tune_table] if tune_table else None),
                   "grid": [wl.n1, wl.n2, wl.n3], "sources": S, "rhs": B, "receivers": R,
                   "setup_s": round(setup_wall, 2),
                   "setup_gpu_pass": setup_gpu,
                   "levels_fwd_max": max(s["levels_fwd"] for s in stats),
                   "n_scc_total": sum(s["n_scc"] for s in stats),
                   "largest_scc": max(s["largest_scc"] for s in stats),
                   "J_ms": round(float(tJ.mean()), 4), "JT_ms": round(float(tT.mean()), 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "vs_sweeping": (round(value / sweep["value"], 2) if sweep and sweep["agrees"] else None),
        "sweeping_baseline": sweep,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
