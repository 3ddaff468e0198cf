"""Solvers and the paired actions J, J^T (oracle; test infrastructure).

J_alpha  = P_alpha A_alpha^{-1} C_alpha              (eq. (source-jacobian), M = I, D = 0)
J_alpha^T y = C_alpha^T A_alpha^{-T} P_alpha^T y      (eq. (source-transpose))
J^T y    = sum_alpha J_alpha^T y_alpha                (Section 4.4, multi-source stacking)

The on-grid source makes D_alpha = 0.  P_alpha samples at the receivers:
a selection for on-grid receivers, or interpolation weights over a few nodes
per receiver; either way it is the explicit sparse matrix OracleOperator.P()
and its transpose scatters and adds.

Three independent solvers for A x = q and A^T y = r:
  * gs_solve      Gauss-Seidel directional sweeping to convergence (Section 3.6),
                  plain C in sweep.c; the transpose sweeps the explicit W^T;
  * dense_solve   LAPACK LU through numpy on tiny grids;
  * superlu_solve scipy's SuperLU on medium grids.
parity: pinned against each other, the 1-D closed form, the adjoint identity,
the scaling identity and the manufactured solution (tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH,
           os.path.join(_HERE, "sweep.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_gs_sweep.restype = ctypes.c_int
        lib.oracle_gs_sweep.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
            ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]
        _lib = lib
    return _lib


def gs_solve(op, Wmat: sp.csr_matrix, q: np.ndarray, max_cycles: int = 10000,
             tol_change: float = 1e-15, tol_res: float = 1e-14, nthreads: int | None = None,
             return_cycles: bool = False):
    """x = q + Wmat x by directional Gauss-Seidel sweeping; q is [N] or [N][B]."""
    lib = _load()
    N = op.N
    q2 = np.asarray(q, dtype=np.float64)
    vec = q2.ndim == 1
    if vec:
        q2 = q2[:, None]
    B = q2.shape[1]
    qT = np.ascontiguousarray(q2.T)
    xT = np.empty_like(qT)
    Wc = Wmat.tocsr()
    rowptr = np.ascontiguousarray(Wc.indptr, dtype=np.int64)
    col = np.ascontiguousarray(Wc.indices, dtype=np.int32)
    val = np.ascontiguousarray(Wc.data, dtype=np.float64)
    cycles = np.zeros(B, dtype=np.int32)
    if nthreads is None:
        nthreads = min(B, os.cpu_count() or 1)
    rc = lib.oracle_gs_sweep(op.dim, op.n1, op.n2, op.n3, rowptr.ctypes.data, col.ctypes.data,
                             val.ctypes.data, B, qT.ctypes.data, xT.ctypes.data, max_cycles,
                             tol_change, tol_res, nthreads, cycles.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_gs_sweep failed: {rc}")
    if np.any(cycles < 0):
        raise RuntimeError(f"Gauss-Seidel sweeping did not converge in {max_cycles} cycles")
    x = np.ascontiguousarray(xT.T)
    if vec:
        x = x[:, 0]
    return (x, cycles) if return_cycles else x


def dense_solve(op, q: np.ndarray, transpose: bool = False) -> np.ndarray:
    """LU of the explicit dense A (tiny grids only)."""
    if op.N > 6000:
        raise ValueError("dense_solve is for tiny grids")
    A = op.A().toarray()
    if transpose:
        A = A.T
    lu = sla.lu_factor(A)
    return sla.lu_solve(lu, q)


_splu_cache = {}


def superlu_solve(op, q: np.ndarray, transpose: bool = False) -> np.ndarray:
    key = id(op)
    ent = _splu_cache.get(key)
    if ent is None or ent[0] is not op:
        _splu_cache.clear()
        ent = (op, spla.splu(op.A().tocsc()))
        _splu_cache[key] = ent
    lu = ent[1]
    return lu.solve(np.asarray(q, dtype=np.float64), trans="T" if transpose else "N")


def _solve(op, q, transpose, solver):
    if solver == "gs":
        return gs_solve(op, op.WT() if transpose else op.W, q)
    if solver == "dense":
        return dense_solve(op, q, transpose)
    if solver == "superlu":
        return superlu_solve(op, q, transpose)
    raise ValueError(solver)


def apply_J(op, ds: np.ndarray, out: str = "nodes", solver: str = "superlu") -> np.ndarray:
    """J ds: q = c * ds, solve A x = q, return x at nodes or receivers."""
    ds = np.asarray(ds, dtype=np.float64)
    q = op.c[:, None] * ds if ds.ndim == 2 else op.c * ds
    x = _solve(op, q, False, solver)
    if out == "nodes":
        return x
    if out == "receivers":
        return op.P() @ x
    raise ValueError(out)


def scatter_receivers(op, y: np.ndarray) -> np.ndarray:
    """P^T y: each receiver value times its weights, added at its nodes."""
    y = np.asarray(y, dtype=np.float64)
    return op.P().T @ y


def apply_JT(op, w: np.ndarray, w_mode: str = "nodes", solver: str = "superlu") -> np.ndarray:
    """J^T w = c * A^{-T} r with r = w (nodes) or P^T w (receivers)."""
    w = np.asarray(w, dtype=np.float64)
    r = w if w_mode == "nodes" else scatter_receivers(op, w)
    lam = _solve(op, r, True, solver)
    return op.c[:, None] * lam if lam.ndim == 2 else op.c * lam


def apply_JT_summed(ops, ws, w_mode: str = "nodes", solver: str = "superlu") -> np.ndarray:
    """sum over sources, in source order, of J_alpha^T w_alpha."""
    acc = None
    for op, w in zip(ops, ws):
        g = apply_JT(op, w, w_mode, solver)
        acc = g if acc is None else acc + g
    return acc
