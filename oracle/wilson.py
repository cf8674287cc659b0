"""ctypes wrapper around the serial FastWalk sampler (``wilson.c``) plus the oracle's own
CSR and integer-CDF construction.  Test infrastructure only.
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson.c")
_LIB = os.path.join(_HERE, "liboracle_wilson.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``wilson.c`` into ``liboracle_wilson.so`` next to it (plain gcc)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_fastwalk.restype = ctypes.c_int
        lib.oracle_fastwalk.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int64, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, P,
                                        ctypes.c_uint64, P, P, P, P, P]
        lib.oracle_fastwalk_stratified.restype = ctypes.c_int
        lib.oracle_fastwalk_stratified.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int64, ctypes.c_uint64,
                                                   ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                                   P, ctypes.c_uint64, P, P, P, P, P]
        lib.oracle_stack_word.restype = ctypes.c_uint64
        lib.oracle_stack_word.argtypes = [ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_random_neighbor_stratified.restype = ctypes.c_int64
        lib.oracle_random_neighbor_stratified.argtypes = [ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P, P, P]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_philox4x32_10.argtypes = [P, P, P]
        lib.oracle_random_neighbor.restype = ctypes.c_int64
        lib.oracle_random_neighbor.argtypes = [ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_uint64, P, P, P]
        lib.oracle_trapwalk.restype = ctypes.c_int
        lib.oracle_trapwalk.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P, P, P]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleCSR:
    """Symmetric CSR with each row sorted by neighbour id; optional integer CDF rows."""

    def __init__(self, n: int, src, dst, w=None):
        src = np.asarray(src, dtype=np.int64)
        dst = np.asarray(dst, dtype=np.int64)
        if src.shape != dst.shape:
            raise ValueError("src/dst length mismatch")
        if np.any(src == dst):
            raise ValueError("self-loop")
        rows = np.concatenate([src, dst])
        cols = np.concatenate([dst, src])
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        if np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
            raise ValueError("duplicate edge")
        self.n = int(n)
        self.row_ptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(self.row_ptr, rows + 1, 1)
        self.row_ptr = np.cumsum(self.row_ptr).astype(np.int64)
        self.col = cols.astype(np.int32)
        if w is None:
            self.cdf = None
            self.weight = np.ones(cols.shape[0])
            self.strength = np.diff(self.row_ptr).astype(np.float64)
        else:
            wf = np.concatenate([np.asarray(w, np.float32), np.asarray(w, np.float32)])[order]
            scaled = wf.astype(np.float64) * float(1 << 24)
            if np.any(scaled != np.floor(scaled)) or np.any(scaled < 1) or np.any(scaled >= 2.0 ** 40):
                raise ValueError("weights must be float32 values in [0.5, 65536)")
            W = scaled.astype(np.uint64)
            self.weight = wf.astype(np.float64)
            # Inclusive prefix sums within each row: a running sum over the whole array
            # (mod 2^64) minus its value just before the row start.
            run = np.cumsum(W, dtype=np.uint64)
            before = np.concatenate([np.zeros(1, np.uint64), run])[self.row_ptr[:-1]]
            deg = np.diff(self.row_ptr)
            self.cdf = run - np.repeat(before, deg)
            totals = self.cdf[self.row_ptr[1:] - 1]
            self.strength = totals.astype(np.float64) / float(1 << 24)
        self.vol = float(self.strength.sum())
        self.pivot = int(np.flatnonzero(self.strength == self.strength.max())[0])


def philox4x32_10(ctr, key) -> tuple[int, int, int, int]:
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return tuple(int(x) for x in o)


def random_neighbor(g: OracleCSR, u: int, k: int, sample: int, graph: int, seed: int, strata: int = 0) -> int:
    """The neighbour chosen at the k-th departure from u in sample `sample` (stack entries
    stratified over samples [0, strata) when strata >= 2)."""
    if strata >= 2:
        return int(_load().oracle_random_neighbor_stratified(u, k, sample, graph, seed, strata, _ptr(g.row_ptr),
                                                             _ptr(g.col), _ptr(g.cdf)))
    return int(_load().oracle_random_neighbor(u, k, sample, graph, seed, _ptr(g.row_ptr), _ptr(g.col),
                                              _ptr(g.cdf)))


def stack_word(k: int, u: int, sample: int, graph: int, seed: int, strata: int = 0) -> int:
    """The 64-bit word of stack entry (u, k) in sample `sample`: the Philox word, or with
    strata >= 2 its Latin-hypercube placement (stratum sigma(sample) of L = strata)."""
    return int(_load().oracle_stack_word(k, u, sample, graph, seed & ((1 << 64) - 1), strata))


def splitmix64(z: int) -> int:
    return int(_load().oracle_splitmix64(ctypes.c_uint64(z & ((1 << 64) - 1))))


def fastwalk_sample(g: OracleCSR, root, seed: int, graph: int, sample_begin: int, nsamples: int,
                    order=None, want_parents: bool = False, threads: int = 1,
                    max_steps: int = (1 << 62), strata: int = 0) -> dict:
    """Run samples [sample_begin, sample_begin + nsamples) serially (or split over threads,
    each thread running a contiguous sample sub-range; sums are integers, so the split does
    not change any output).  `root` is one node (a rooted spanning tree per sample) or a
    sequence of distinct nodes (a spanning forest rooted at that set).  strata >= 2 stratifies
    every stack entry over samples [0, strata) (Latin hypercube), which must hold the run."""
    lib = _load()
    n = g.n
    roots = np.ascontiguousarray(np.atleast_1d(np.asarray(root, dtype=np.int64)))
    if roots.size != np.unique(roots).size:
        raise ValueError("the root set lists a node twice")
    visits = np.zeros(n, dtype=np.uint64)
    visits_sq = np.zeros(n, dtype=np.uint64)
    steps = np.zeros(nsamples, dtype=np.uint64)
    hsh = np.zeros(nsamples, dtype=np.uint64)
    parents = np.zeros((nsamples, n), dtype=np.int32) if want_parents else None
    ordr = None if order is None else np.ascontiguousarray(order, dtype=np.int32)

    def run(lo, hi):
        v = np.zeros(n, dtype=np.uint64)
        v2 = np.zeros(n, dtype=np.uint64)
        par = parents[lo:hi] if parents is not None else None
        rc = lib.oracle_fastwalk_stratified(n, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.cdf), _ptr(roots), roots.size,
                                            seed, graph, sample_begin + lo, hi - lo, strata, _ptr(ordr), max_steps,
                                            _ptr(v), _ptr(v2), _ptr(steps[lo:hi]), _ptr(hsh[lo:hi]), _ptr(par))
        if rc != 0:
            raise RuntimeError(f"oracle_fastwalk failed with code {rc}")
        return v, v2

    if threads <= 1 or nsamples < 2:
        parts = [run(0, nsamples)]
    else:
        bounds = np.linspace(0, nsamples, min(threads, nsamples) + 1).astype(int)
        with cf.ThreadPoolExecutor(max_workers=len(bounds) - 1) as ex:
            parts = list(ex.map(lambda ab: run(*ab), zip(bounds[:-1], bounds[1:])))
    for v, v2 in parts:
        visits += v
        visits_sq += v2
    return {"visits": visits, "visits_sq": visits_sq, "steps": steps, "hash": hsh, "parents": parents}


def trapwalk_sample(g: OracleCSR, v: int, seed: int, graph: int, walk_begin: int, nwalks: int, threads: int = 1,
                    max_steps: int = (1 << 62)) -> dict:
    """Walks [walk_begin, walk_begin + nwalks) from every node u != v, each stopped at the trap v
    and counting its visits to u (Lemma 5.1); split over threads by walk range (integer sums,
    so the split changes nothing).  Returns visits, visits_sq [n] and the total steps."""
    lib = _load()
    n = g.n

    def run(lo, hi):
        a = np.zeros(n, dtype=np.uint64)
        b = np.zeros(n, dtype=np.uint64)
        st = np.zeros(1, dtype=np.uint64)
        rc = lib.oracle_trapwalk(n, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.cdf), v, seed, graph, walk_begin + lo,
                                 hi - lo, max_steps, _ptr(a), _ptr(b), _ptr(st))
        if rc != 0:
            raise RuntimeError(f"oracle_trapwalk failed with code {rc}")
        return a, b, int(st[0])

    if threads <= 1 or nwalks < 2:
        parts = [run(0, nwalks)]
    else:
        bounds = np.linspace(0, nwalks, min(threads, nwalks) + 1).astype(int)
        with cf.ThreadPoolExecutor(max_workers=len(bounds) - 1) as ex:
            parts = list(ex.map(lambda ab: run(*ab), zip(bounds[:-1], bounds[1:])))
    return {"visits": sum(p[0] for p in parts), "visits_sq": sum(p[1] for p in parts),
            "steps": sum(p[2] for p in parts)}
