"""ctypes wrapper around the serial FastChol oracle (``fastchol.c``): Section 4, Algorithm 2.
Test infrastructure only.

``fastchol(n, src, dst, w, v, ...)`` forms the grounded normalised Laplacian calL_v of the graph
(node v removed, the remaining nodes in the given elimination order), factors it with IChol,
builds the windowed, sparsified inverse columns, and returns tau~ (the estimate of
diag(calL_v^{-1}) for every node, 0 at v) together with the factor and per-column sizes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fastchol.c")
_LIB = os.path.join(_HERE, "liboracle_fastchol.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``fastchol.c`` into ``liboracle_fastchol.so`` next to it (plain gcc)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_ichol.restype = ctypes.c_int
        lib.oracle_ichol.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, ctypes.POINTER(P),
                                     ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_sparse_inverse.restype = ctypes.c_int
        lib.oracle_sparse_inverse.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int64, ctypes.c_double, P, P]
        lib.oracle_sparse_inverse_dump.restype = ctypes.c_int
        lib.oracle_sparse_inverse_dump.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_int64, ctypes.c_double, P, ctypes.c_int64, P, P, P]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def grounded_normalized_lower(n: int, src, dst, w, v: int, order=None):
    """calL_v = I - D^{-1/2} A D^{-1/2} without row and column v, its rows and columns in
    elimination order (`order`: the nodes other than v, first to last; default ascending ids),
    as the lower triangle in compressed columns (diagonal first, rows ascending).  Returns
    (ptr, row, val, nodes) with nodes[j] the node of column j."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    wt = np.ones(src.shape[0]) if w is None else np.asarray(w, np.float64)
    d = np.zeros(n)
    np.add.at(d, src, wt)
    np.add.at(d, dst, wt)
    nodes = np.array([u for u in range(n) if u != v], np.int64) if order is None else np.asarray(order, np.int64)
    if nodes.shape[0] != n - 1 or np.any(nodes == v) or np.unique(nodes).shape[0] != n - 1:
        raise ValueError("order must list every node but v once")
    pos = -np.ones(n, np.int64)
    pos[nodes] = np.arange(n - 1)
    keep = (src != v) & (dst != v)
    a, b, x = pos[src[keep]], pos[dst[keep]], -wt[keep] / np.sqrt(d[src[keep]] * d[dst[keep]])
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    N = n - 1
    rows = np.concatenate([np.arange(N), hi])
    cols = np.concatenate([np.arange(N), lo])
    vals = np.concatenate([np.ones(N), x])
    o = np.lexsort((rows, cols))
    rows, cols, vals = rows[o], cols[o], vals[o]
    ptr = np.zeros(N + 1, np.int64)
    np.add.at(ptr, cols + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int64)
    return ptr, rows.astype(np.int64), vals.astype(np.float64), nodes


def ichol(ptr, row, val, droptol: float):
    """IChol of the lower-triangular CSC (ptr, row, val): returns (r_ptr, r_row, r_val)."""
    lib = _load()
    N = ptr.shape[0] - 1
    r_ptr = np.zeros(N + 1, np.int64)
    prow, pval = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    rc = lib.oracle_ichol(N, _ptr(np.ascontiguousarray(ptr, np.int64)), _ptr(np.ascontiguousarray(row, np.int64)),
                          _ptr(np.ascontiguousarray(val, np.float64)), float(droptol), _ptr(r_ptr),
                          ctypes.byref(prow), ctypes.byref(pval), ctypes.byref(nnz))
    if rc != 0:
        raise RuntimeError(f"oracle_ichol failed with code {rc}")
    k = nnz.value
    r_row = np.ctypeslib.as_array(ctypes.cast(prow, ctypes.POINTER(ctypes.c_int64)), shape=(k,)).copy()
    r_val = np.ctypeslib.as_array(ctypes.cast(pval, ctypes.POINTER(ctypes.c_double)), shape=(k,)).copy()
    lib.oracle_free(prow)
    lib.oracle_free(pval)
    return r_ptr, r_row, r_val


def sparse_inverse(r_ptr, r_row, r_val, deg, ws: float, zeta: int, eps_p: float):
    """Algorithm 2's loop: tau~[N] and the kept entries per column."""
    lib = _load()
    N = r_ptr.shape[0] - 1
    tau = np.zeros(N)
    snz = np.zeros(N, np.int64)
    deg = np.ascontiguousarray(deg, np.float64)
    rc = lib.oracle_sparse_inverse(N, _ptr(r_ptr), _ptr(r_row), _ptr(r_val), _ptr(deg), float(deg.max()), float(ws),
                                   int(zeta), float(eps_p), _ptr(tau), _ptr(snz))
    if rc != 0:
        raise RuntimeError(f"oracle_sparse_inverse failed with code {rc}")
    return tau, snz


def sparse_inverse_columns(r_ptr, r_row, r_val, deg, ws: float, zeta: int, eps_p: float, cap: int = 1 << 24):
    """Algorithm 2's loop, returning tau~ and S~ itself as a CSC (s_ptr, s_row, s_val)."""
    lib = _load()
    N = r_ptr.shape[0] - 1
    tau = np.zeros(N)
    s_ptr = np.zeros(N + 1, np.int64)
    s_row = np.zeros(cap, np.int64)
    s_val = np.zeros(cap)
    deg = np.ascontiguousarray(deg, np.float64)
    rc = lib.oracle_sparse_inverse_dump(N, _ptr(r_ptr), _ptr(r_row), _ptr(r_val), _ptr(deg), float(deg.max()),
                                        float(ws), int(zeta), float(eps_p), _ptr(tau), cap, _ptr(s_ptr), _ptr(s_row),
                                        _ptr(s_val))
    if rc != 0:
        raise RuntimeError(f"oracle_sparse_inverse_dump failed with code {rc}")
    k = int(s_ptr[-1])
    return tau, s_ptr, s_row[:k].copy(), s_val[:k].copy()


def fastchol(n: int, src, dst, w, v: int, droptol: float = 1e-4, ws: float = 16, zeta: int = 16,
             eps_p: float = 1e-3, order=None) -> dict:
    """FastChol's estimate of diag(calL_v^{-1}) for every node (0 at v)."""
    ptr, row, val, nodes = grounded_normalized_lower(n, src, dst, w, v, order)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    wt = np.ones(src.shape[0]) if w is None else np.asarray(w, np.float64)
    d = np.zeros(n)
    np.add.at(d, src, wt)
    np.add.at(d, dst, wt)
    r_ptr, r_row, r_val = ichol(ptr, row, val, droptol)
    tau_c, snz = sparse_inverse(r_ptr, r_row, r_val, d[nodes], ws, zeta, eps_p)
    tau = np.zeros(n)
    tau[nodes] = tau_c
    return {"tau": tau, "r_ptr": r_ptr, "r_row": r_row, "r_val": r_val, "s_nnz": snz, "nodes": nodes}
