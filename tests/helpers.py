"""Shared helpers of the GPU tests: run the library through the C ABI on
seeded inputs and compute the oracle's answer for the same inputs."""
from __future__ import annotations

import numpy as np

import oracle as O
import workloads as W
from oracle.assembly import assemble_workload


def rel_l2_pairs(x, ref):
    """max over (source, rhs) pairs of ||x - ref||_2 / ||ref||_2; arrays [S][*][B]."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sqrt(np.sum((x - ref) ** 2, axis=-2))
    den = np.sqrt(np.sum(ref ** 2, axis=-2))
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den))


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def states_for(fm, wl, S=None):
    S = wl.S if S is None else S
    return fm.build_frozen_states(wl.dim, wl.n1, wl.n2, wl.n3, wl.G, wl.T[:S], wl.s, wl.src[:S],
                                  wl.rcv, nthreads=8, rcv_weights=getattr(wl, "rcv_w", None),
                                  stencil=getattr(wl, "stencil", 6))


def oracle_ops(wl, S=None):
    S = wl.S if S is None else S
    return [assemble_workload(wl, a) for a in range(S)]


def oracle_J(ops, ds, per_pair, out="nodes", solver="superlu"):
    res = []
    for a, op in enumerate(ops):
        d = ds[a] if per_pair else ds
        res.append(O.apply_J(op, d, out, solver))
    return np.stack(res)


def oracle_JT(ops, w, w_mode="nodes", solver="superlu"):
    return np.stack([O.apply_JT(op, w[a], w_mode, solver) for a, op in enumerate(ops)])


def gpu_run(fm, torch, states, B, prec, direction, inp, in_mode, out_mode, tuning=None):
    """One apply through the C ABI; returns a numpy copy of the output."""
    dev = torch.device("cuda:0")
    dt = torch.float64 if prec == fm.FM_FP64 else torch.float32
    batch = fm.Batch(states, B, prec, tuning=tuning)
    S, N, R = batch.S, batch.N, batch.R
    x = torch.from_numpy(np.ascontiguousarray(inp)).to(dev, dt)
    if direction == "J":
        shape = (S, N, B) if out_mode == fm.FM_OUT_NODES else (S, R, B)
        out = torch.full(shape, float("nan"), device=dev, dtype=dt)
        batch.apply_J(x, in_mode, out, out_mode)
    else:
        shape = (S, N, B) if out_mode == fm.FM_JT_PER_SOURCE else (N, B)
        out = torch.full(shape, float("nan"), device=dev, dtype=dt)
        batch.apply_JT(x, in_mode, out, out_mode)
    batch.status()
    res = out.cpu().numpy().astype(np.float64)
    batch.free()
    return res


def seeded_ds(wl, B, seed, S=None, per_pair=True):
    rng = np.random.default_rng(seed)
    S = wl.S if S is None else S
    if per_pair:
        return np.stack([W.smooth_noise(wl, B, rng) for _ in range(S)])
    return W.smooth_noise(wl, B, rng)
