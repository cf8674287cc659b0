"""Python binding of the FastWalk library: torch tensors in, torch tensors out.

PyTorch supplies device memory (inputs, outputs and the workspaces the library asks for) and
the current HIP stream; the computation itself runs in librwc.so.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (BackwardParams, BatchTuneResult, FastcholParams, RwcCsr, SampleOutputs, SampleParams, SolveParams,
                   TrapParams,
                   TuneResult, check)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p | None:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_tensor(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(device)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Graph:
    """An undirected graph built on the device by rwc_build_csr_ex.  allow_disconnected=True
    accepts several connected components (RWC_BUILD_ALLOW_DISCONNECTED): such a graph is for
    forests rooted at a set that meets every component and the group estimate; the pivot
    estimate, trap walks, FastChol, the adjoint and unrooted sampling refuse it."""

    def __init__(self, n: int, src, dst, w=None, device: str | torch.device = "cuda", allow_disconnected: bool = False):
        L = _lib.lib()
        self.device = torch.device(device)
        self.src = _dev_tensor(src, torch.int32, self.device)
        self.dst = _dev_tensor(dst, torch.int32, self.device)
        self.w = None if w is None else _dev_tensor(w, torch.float32, self.device)
        self.n = int(n)
        self.m = int(self.src.numel())
        size = ctypes.c_size_t()
        check(L.rwc_build_csr_workspace(self.n, self.m, int(self.w is not None), ctypes.byref(size)),
              "rwc_build_csr_workspace")
        self.ws = _workspace(size.value, self.device)
        self.csr = RwcCsr()
        flags = _lib.RWC_BUILD_ALLOW_DISCONNECTED if allow_disconnected else 0
        check(L.rwc_build_csr_ex(self.n, self.m, _ptr(self.src), _ptr(self.dst), _ptr(self.w), flags, _ptr(self.ws),
                                 self.ws.numel(), ctypes.byref(self.csr), _stream()), "rwc_build_csr_ex")

    # -- views of the device CSR (for tests and diagnostics), in the graph's internal order:
    # node_id()[x] is the input id of internal index x --
    def _view(self, addr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        off = addr - self.ws.data_ptr()
        nbytes = count * torch.empty(0, dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    @property
    def pivot(self) -> int:
        return int(self.csr.pivot)

    @property
    def vol(self) -> float:
        return float(self.csr.vol)

    @property
    def nnz(self) -> int:
        return int(self.csr.nnz)

    def row_ptr(self) -> torch.Tensor:
        return self._view(self.csr.row_ptr, self.n + 1, torch.int32)

    def col(self) -> torch.Tensor:
        return self._view(self.csr.col, self.nnz, torch.int32)

    def weight(self) -> torch.Tensor:
        return self._view(self.csr.weight, self.nnz, torch.float32)

    def edge_id(self) -> torch.Tensor:
        return self._view(self.csr.edge_id, self.nnz, torch.int32)

    def cdf(self) -> torch.Tensor | None:
        if not self.csr.cdf:
            return None
        return self._view(self.csr.cdf, self.nnz, torch.int64)  # bit pattern of uint64

    def strength(self) -> torch.Tensor:
        return self._view(self.csr.strength, self.n, torch.float64)

    def bfs_order(self) -> torch.Tensor:
        return self._view(self.csr.bfs_order, self.n, torch.int32)

    def node_id(self) -> torch.Tensor:
        return self._view(self.csr.node_id, self.n, torch.int32)

    def node_index(self) -> torch.Tensor:
        return self._view(self.csr.node_index, self.n, torch.int32)

    @property
    def internal_order(self) -> int:
        return int(self.csr.internal_order)

    @property
    def components(self) -> int:
        return int(self.csr.components)

    def component(self) -> torch.Tensor:
        """[n] by input id: the smallest input id of each node's connected component."""
        return self._view(self.csr.component, self.n, torch.int32)

    def rec(self) -> torch.Tensor:
        return self._view(self.csr.rec, 16 * self.n, torch.int32)


def _sample_setup(gl, num_samples, seed, sample_begin, root, trees_in_flight, walkers_per_tree, persistent,
                  capture, accumulate, max_steps_per_tree, graph_index_base, bfs_starts, starts, path_ring, roots,
                  lds_state=None, walkers_per_graph=None, strata=0):
    arr = (RwcCsr * len(gl))(*[g.csr for g in gl])
    flags = 0
    if persistent:
        flags |= _lib.RWC_SAMPLE_PERSISTENT
    if capture:
        flags |= _lib.RWC_SAMPLE_GRAPH_CAPTURE
    if accumulate:
        flags |= _lib.RWC_SAMPLE_ACCUMULATE
    if bfs_starts is not None:
        flags |= _lib.RWC_SAMPLE_BFS_STARTS if bfs_starts else _lib.RWC_SAMPLE_ID_STARTS
    if starts == "spread":
        flags |= _lib.RWC_SAMPLE_SPREAD_STARTS
    elif starts == "shared":
        flags |= _lib.RWC_SAMPLE_SHARED_STARTS
    elif starts != "auto":
        raise ValueError(f"starts must be 'auto', 'shared' or 'spread', not {starts!r}")
    if path_ring is not None:
        flags |= _lib.RWC_SAMPLE_PATH_RING if path_ring else _lib.RWC_SAMPLE_NO_PATH_RING
    if lds_state is False:
        flags |= _lib.RWC_SAMPLE_NO_LDS_STATE
    p = SampleParams(seed=seed, sample_begin=sample_begin, num_samples=num_samples, root=root, flags=flags,
                     trees_in_flight=trees_in_flight, walkers_per_tree=walkers_per_tree,
                     max_steps_per_tree=max_steps_per_tree, graph_index_base=graph_index_base,
                     strata=int(strata))
    if roots is not None:
        p.roots = roots.data_ptr()
        p.num_roots = roots.numel()
    if walkers_per_graph is not None:
        wpg = (ctypes.c_int32 * len(gl))(*[int(x) for x in walkers_per_graph])
        p.walkers_per_graph = ctypes.cast(wpg, ctypes.c_void_p)
        p._keep = wpg   # the host array must live as long as the params
    return arr, p


def _roots_tensor(roots, device):
    if roots is None:
        return None
    return _dev_tensor(roots, torch.int32, device)


def sample_forests(graphs: Graph | Sequence[Graph], num_samples: int, seed: int, sample_begin: int = 0,
                   root: int = -1, trees_in_flight: int = 0, walkers_per_tree: int = 0,
                   persistent: bool = False, capture: bool = False, want_sq: bool = True,
                   want_hash: bool = True, dump: Sequence[int] = (), max_steps_per_tree: int = 0,
                   graph_index_base: int = 0, accumulate: dict | None = None,
                   workspace: torch.Tensor | None = None, timing: bool = False,
                   bfs_starts: bool | None = None, starts: str = "auto", path_ring: bool | None = None,
                   roots=None, sync: bool = True, out: dict | None = None, lds_state: bool | None = None,
                   walkers_per_graph: Sequence[int] | None = None, strata: int = 0) -> dict:
    """Samples `num_samples` rooted spanning trees of every graph (rwc_sample_forests).

    Returns device tensors: counts [sum n] (int64 holding uint64 values), counts_sq,
    total_steps [G], tree_hash [G, num_samples], parents [len(dump), n] and the workspace
    used (pass it back as `workspace` to reuse it).  With timing=True also walk_ms and
    reduce_ms: device time of the walk and reduction kernels (hipEvents on the stream).
    `starts` ("auto", "shared", "spread"), `bfs_starts` (None = automatic, True =
    breadth-first from the root, False = ascending ids) and `path_ring` (None = automatic) pick
    how walker teams schedule their walks, and lds_state=False keeps every tree's state in HBM
    (by default small graphs grow their trees in LDS); the forest does not depend on them.  `roots` (ids,
    single graph) samples spanning forests rooted at that set instead of trees rooted at one
    node.  `out` (a dict returned by an earlier call) reuses its output tensors, so that a
    repeated call with capture=True replays the library's cached hipGraph.  The call is
    stream-ordered; with sync=True (default) it then waits and raises on a device-side error
    (rwc_workspace_status).  strata = L >= 2 stratifies every stack entry over samples
    [0, L) (Latin hypercube), a lower-variance estimate at equal trees; the call's samples
    must lie in that range."""
    L = _lib.lib()
    gl = [graphs] if isinstance(graphs, Graph) else list(graphs)
    G = len(gl)
    dev = gl[0].device
    rt = _roots_tensor(roots, dev)
    arr, p = _sample_setup(gl, num_samples, seed, sample_begin, root, trees_in_flight, walkers_per_tree, persistent,
                           capture, accumulate is not None, max_steps_per_tree, graph_index_base, bfs_starts, starts,
                           path_ring, rt, lds_state, walkers_per_graph, strata)
    size = ctypes.c_size_t()
    check(L.rwc_sample_forests_workspace(arr, G, ctypes.byref(p), ctypes.byref(size)),
          "rwc_sample_forests_workspace")
    if workspace is None or workspace.numel() < size.value:
        workspace = _workspace(size.value, dev)
    total = sum(g.n for g in gl)
    if accumulate is not None:
        res = accumulate
    elif out is not None:
        res = out
    else:
        res = {
            "counts": torch.empty(total, dtype=torch.int64, device=dev),
            "counts_sq": torch.empty(total, dtype=torch.int64, device=dev) if want_sq else None,
            "total_steps": torch.empty(G, dtype=torch.int64, device=dev),
        }
    th = res.get("tree_hash")
    if not want_hash:
        res["tree_hash"] = None
    elif th is None or tuple(th.shape) != (G, num_samples):
        res["tree_hash"] = torch.empty((G, num_samples), dtype=torch.int64, device=dev)
    dump = list(dump)
    pa = res.get("parents")
    if not dump:
        res["parents"] = None
    elif pa is None or tuple(pa.shape) != (len(dump), gl[0].n):
        res["parents"] = torch.empty((len(dump), gl[0].n), dtype=torch.int32, device=dev)
    dump_host = (ctypes.c_int64 * max(1, len(dump)))(*dump) if dump else None
    so = SampleOutputs(counts=_ptr(res["counts"]), counts_sq=_ptr(res.get("counts_sq")),
                       total_steps=_ptr(res.get("total_steps")), tree_hash=_ptr(res["tree_hash"]),
                       parents=_ptr(res["parents"]),
                       dump_samples=ctypes.cast(dump_host, ctypes.c_void_p) if dump else None,
                       ndump=len(dump))
    tms = (ctypes.c_float * 2)()
    if timing:
        so.timing_ms = ctypes.cast(tms, ctypes.c_void_p)
    plan = (ctypes.c_int32 * 8)()
    so.plan = ctypes.cast(plan, ctypes.c_void_p)
    check(L.rwc_sample_forests(arr, G, ctypes.byref(p), ctypes.byref(so), _ptr(workspace), workspace.numel(),
                               _stream()), "rwc_sample_forests")
    if sync and not timing:
        check(L.rwc_workspace_status(_ptr(workspace), _stream()), "rwc_sample_forests (device status)")
    res["workspace"] = workspace
    res["roots"] = rt
    res["walkers_per_tree"], res["trees_in_flight"], res["batches"] = int(plan[0]), int(plan[1]), int(plan[2])
    kernels = (("wilson_walk", "wilson_team<false>", "wilson_team<true>", "wilson_team_lds<false>",
                "wilson_team_lds<true>") if strata < 2 else
               ("wilson_walk_strata", "wilson_team_strata<false>", "wilson_team_strata<true>",
                "wilson_team_lds_strata<false>", "wilson_team_lds_strata<true>"))
    res["walk_kernel"] = kernels[int(plan[3])]
    res["lds_graphs"] = int(plan[7])
    res["starts"] = "spread" if plan[4] else "shared"
    res["start_order"] = "breadth-first" if plan[5] else "ascending"
    res["graph_replayed"] = int(plan[6])
    if timing:
        res["walk_ms"], res["reduce_ms"] = float(tms[0]), float(tms[1])
    return res


def prepare_sampling(graphs: Graph | Sequence[Graph], num_samples: int, workspace: torch.Tensor | None = None,
                     roots=None, **kw) -> dict:
    """rwc_sample_prepare: writes the argument tables of a sampling call into its workspace so
    that sample_forests(..., workspace=...) with the same graphs and parameters (seed and
    sample_begin may differ) can run on a stream that is being captured into a hipGraph.
    Returns {"workspace": ..., "roots": ...}; pass both back."""
    L = _lib.lib()
    gl = [graphs] if isinstance(graphs, Graph) else list(graphs)
    dev = gl[0].device
    rt = _roots_tensor(roots, dev)
    arr, p = _sample_setup(gl, num_samples, kw.get("seed", 0), kw.get("sample_begin", 0), kw.get("root", -1),
                           kw.get("trees_in_flight", 0), kw.get("walkers_per_tree", 0), kw.get("persistent", False),
                           False, kw.get("accumulate", False), kw.get("max_steps_per_tree", 0),
                           kw.get("graph_index_base", 0), kw.get("bfs_starts"), kw.get("starts", "auto"),
                           kw.get("path_ring"), rt, kw.get("lds_state"), kw.get("walkers_per_graph"),
                           kw.get("strata", 0))
    size = ctypes.c_size_t()
    check(L.rwc_sample_forests_workspace(arr, len(gl), ctypes.byref(p), ctypes.byref(size)),
          "rwc_sample_forests_workspace")
    if workspace is None or workspace.numel() < size.value:
        workspace = _workspace(size.value, dev)
    check(L.rwc_sample_prepare(arr, len(gl), ctypes.byref(p), _ptr(workspace), workspace.numel(), _stream()),
          "rwc_sample_prepare")
    return {"workspace": workspace, "roots": rt}


def workspace_status(workspace: torch.Tensor) -> None:
    """Waits for the stream and raises if the last stream-ordered call on `workspace` reported
    a device-side error."""
    check(_lib.lib().rwc_workspace_status(_ptr(workspace), _stream()), "rwc_workspace_status")


def release_cached_graphs() -> None:
    _lib.lib().rwc_release_cached_graphs()


def sample_trap_walks(graph: Graph, num_walks: int, seed: int, walk_begin: int = 0, trap: int = -1,
                      graph_index: int = 0, max_steps_per_walk: int = 0, want_sq: bool = True,
                      sync: bool = True) -> dict:
    """Trap walks (rwc_sample_trap_walks): num_walks walks from every node u != trap (default the
    pivot), each stopped at the trap and counting its visits to u.  Returns counts [n],
    counts_sq [n] and total_steps [1] (int64 tensors holding uint64 values): counts / l
    estimates the same diagonal as the Wilson forests, so estimate(graph, counts, num_walks)
    gives RWC."""
    L = _lib.lib()
    dev = graph.device
    p = TrapParams(seed=seed, walk_begin=walk_begin, num_walks=num_walks, trap=trap, graph_index=graph_index,
                   max_steps_per_walk=max_steps_per_walk)
    size = ctypes.c_size_t()
    check(L.rwc_sample_trap_walks_workspace(ctypes.byref(graph.csr), ctypes.byref(p), ctypes.byref(size)),
          "rwc_sample_trap_walks_workspace")
    ws = _workspace(size.value, dev)
    res = {"counts": torch.empty(graph.n, dtype=torch.int64, device=dev),
           "counts_sq": torch.empty(graph.n, dtype=torch.int64, device=dev) if want_sq else None,
           "total_steps": torch.empty(1, dtype=torch.int64, device=dev)}
    check(L.rwc_sample_trap_walks(ctypes.byref(graph.csr), ctypes.byref(p), _ptr(res["counts"]),
                                  _ptr(res["counts_sq"]), _ptr(res["total_steps"]), _ptr(ws), ws.numel(), _stream()),
          "rwc_sample_trap_walks")
    if sync:
        check(L.rwc_workspace_status(_ptr(ws), _stream()), "rwc_sample_trap_walks (device status)")
    res["workspace"] = ws
    return res


def autotune(graph: Graph, num_samples: int, seed: int, sample_begin: int = 0,
             budget_bytes: int = 64 << 30) -> dict:
    """Times one batch of each candidate (walkers per tree and trees in flight, then the team
    schedule) and returns the fastest (rwc_autotune_sampler); cached per graph class for the
    process.  `path_ring`, `starts` and `bfs_starts` are the winner's schedule in the form
    sample_forests takes (None / "auto" when the automatic schedule won)."""
    L = _lib.lib()
    p = SampleParams(seed=seed, sample_begin=sample_begin, num_samples=num_samples, root=-1)
    size = ctypes.c_size_t()
    check(L.rwc_autotune_workspace(ctypes.byref(graph.csr), ctypes.byref(p), int(budget_bytes), ctypes.byref(size)),
          "rwc_autotune_workspace")
    ws = _workspace(size.value, graph.device)
    r = TuneResult()
    check(L.rwc_autotune_sampler(ctypes.byref(graph.csr), ctypes.byref(p), int(budget_bytes), ctypes.byref(r),
                                 _ptr(ws), ws.numel(), _stream()), "rwc_autotune_sampler")
    def pick(on, off, yes, no, neither):
        return yes if r.flags & on else (no if r.flags & off else neither)
    return {"walkers_per_tree": r.walkers_per_tree, "trees_in_flight": r.trees_in_flight,
            "steps_per_s": r.steps_per_s, "candidates": r.candidates, "cached": bool(r.cached),
            "path_ring": pick(_lib.RWC_SAMPLE_PATH_RING, _lib.RWC_SAMPLE_NO_PATH_RING, True, False, None),
            "starts": pick(_lib.RWC_SAMPLE_SPREAD_STARTS, _lib.RWC_SAMPLE_SHARED_STARTS, "spread", "shared", "auto"),
            "bfs_starts": pick(_lib.RWC_SAMPLE_BFS_STARTS, _lib.RWC_SAMPLE_ID_STARTS, True, False, None),
            "lds_state": False if r.flags & _lib.RWC_SAMPLE_NO_LDS_STATE else None}


def autotune_batch(graphs: Sequence[Graph], num_samples: int, seed: int, sample_begin: int = 0) -> dict:
    """rwc_autotune_batch: walkers per tree for the mesh-like graphs and for the others, then the
    schedule, timed on probes of the whole batch.  Returns the choice in the form sample_forests
    takes (walkers_per_graph, path_ring, bfs_starts, lds_state) plus the probe statistics."""
    L = _lib.lib()
    gl = list(graphs)
    arr = (RwcCsr * len(gl))(*[g.csr for g in gl])
    p = SampleParams(seed=seed, sample_begin=sample_begin, num_samples=num_samples, root=-1,
                     flags=_lib.RWC_SAMPLE_PERSISTENT)
    size = ctypes.c_size_t()
    check(L.rwc_autotune_batch_workspace(arr, len(gl), ctypes.byref(p), ctypes.byref(size)),
          "rwc_autotune_batch_workspace")
    ws = _workspace(size.value, gl[0].device)
    r = BatchTuneResult()
    check(L.rwc_autotune_batch(arr, len(gl), ctypes.byref(p), ctypes.byref(r), _ptr(ws), ws.numel(), _stream()),
          "rwc_autotune_batch")
    del ws
    wpg = [r.walkers_mesh if int(g.csr.bfs_depth) > 32 else r.walkers_other for g in gl]
    return {"walkers_mesh": r.walkers_mesh, "walkers_other": r.walkers_other, "walkers_per_graph": wpg,
            "path_ring": bool(r.flags & _lib.RWC_SAMPLE_PATH_RING),
            "bfs_starts": bool(r.flags & _lib.RWC_SAMPLE_BFS_STARTS),
            "lds_state": False if r.flags & _lib.RWC_SAMPLE_NO_LDS_STATE else None,
            "flags": int(r.flags), "candidates": r.candidates, "steps_per_s": r.steps_per_s,
            "probe_samples": r.probe_samples, "cached": bool(r.cached)}


def estimate(graph: Graph, counts: torch.Tensor, l: int, counts_sq: torch.Tensor | None = None,
             tol: float = 1e-12, max_iter: int = 0, want_hit: bool = True, want_stderr: bool = False,
             stream_ordered: bool = False, workspace: torch.Tensor | None = None, out: dict | None = None) -> dict:
    """RWC from visit totals (rwc_estimate): returns rwc, hit (hitting times to the pivot),
    stderr and the CG iteration count.  stream_ordered=True enqueues max_iter iterations that
    stop on the device (no host synchronisation; capturable): iters is then -1 and the outcome
    is read with workspace_status(res["workspace"])."""
    L = _lib.lib()
    dev = graph.device
    size = ctypes.c_size_t()
    check(L.rwc_estimate_workspace(ctypes.byref(graph.csr), ctypes.byref(size)), "rwc_estimate_workspace")
    ws = workspace if workspace is not None and workspace.numel() >= size.value else _workspace(size.value, dev)
    if out is None:
        out = {"rwc": torch.empty(graph.n, dtype=torch.float64, device=dev),
               "hit": torch.empty(graph.n, dtype=torch.float64, device=dev) if want_hit else None,
               "stderr": torch.empty(graph.n, dtype=torch.float64, device=dev) if want_stderr else None}
    sp = SolveParams(tol=tol, max_iter=max_iter, check_every=_lib.RWC_SOLVE_STREAM_ORDERED if stream_ordered else 0)
    iters = ctypes.c_int32()
    check(L.rwc_estimate(ctypes.byref(graph.csr), _ptr(counts), _ptr(counts_sq), int(l), ctypes.byref(sp),
                         _ptr(out["rwc"]), _ptr(out.get("hit")), _ptr(out.get("stderr")), ctypes.byref(iters),
                         _ptr(ws), ws.numel(), _stream()),
          "rwc_estimate")
    return {**out, "iters": iters.value, "workspace": ws}


def estimate_diag(graph: Graph, diag: torch.Tensor, tol: float = 1e-12, max_iter: int = 0,
                  want_hit: bool = True) -> dict:
    """RWC from an estimate of diag(calL_v^{-1}) by input id (FastChol's tau~): rwc_estimate_diag."""
    L = _lib.lib()
    dev = graph.device
    size = ctypes.c_size_t()
    check(L.rwc_estimate_workspace(ctypes.byref(graph.csr), ctypes.byref(size)), "rwc_estimate_workspace")
    ws = _workspace(size.value, dev)
    rwc = torch.empty(graph.n, dtype=torch.float64, device=dev)
    hit = torch.empty(graph.n, dtype=torch.float64, device=dev) if want_hit else None
    sp = SolveParams(tol=tol, max_iter=max_iter, check_every=0)
    iters = ctypes.c_int32()
    check(L.rwc_estimate_diag(ctypes.byref(graph.csr), _ptr(diag), ctypes.byref(sp), _ptr(rwc), _ptr(hit),
                              ctypes.byref(iters), _ptr(ws), ws.numel(), _stream()), "rwc_estimate_diag")
    return {"rwc": rwc, "hit": hit, "iters": iters.value}


FASTCHOL_METHODS = {"auto": _lib.RWC_FASTCHOL_AUTO, "chain": _lib.RWC_FASTCHOL_CHAIN,
                    "dense": _lib.RWC_FASTCHOL_DENSE}


def fastchol(graph: Graph, droptol: float = 1e-4, window: float = 16.0, zeta: int = 16, eps_p: float = 1e-3,
             factor_capacity: int | None = None, inverse_capacity: int | None = None, sync: bool = True,
             method: str = "auto") -> dict:
    """FastChol's tau~ (rwc_fastchol): the estimate of diag(calL_v^{-1}) by input id from the
    threshold incomplete Cholesky factor and its windowed, sparsified inverse (Section 4,
    Algorithm 2).  The pools default to 512 (n - 1) entries each for the factor and for S~, at
    most a full triangle.  method: "dense" (right-looking IChol on the packed (n-1) n / 2 triangle), "chain"
    (left-looking on one wave) or "auto" (dense up to 32 GiB); both give the same bits.  With
    sync=True waits, raises on a device-side error and also returns the number of entries of
    the factor and of S~."""
    L = _lib.lib()
    dev = graph.device
    n1 = graph.n - 1
    tri = n1 * (n1 + 1) // 2
    if method not in FASTCHOL_METHODS:
        raise ValueError(f"method must be one of {sorted(FASTCHOL_METHODS)}")
    p = FastcholParams(droptol=float(droptol), window=float(window), eps_p=float(eps_p), zeta=int(zeta),
                       method=FASTCHOL_METHODS[method],
                       factor_capacity=int(factor_capacity if factor_capacity is not None else min(512 * n1, tri)),
                       inverse_capacity=int(inverse_capacity if inverse_capacity is not None else min(512 * n1, tri)))
    size = ctypes.c_size_t()
    check(L.rwc_fastchol_workspace(ctypes.byref(graph.csr), ctypes.byref(p), ctypes.byref(size)),
          "rwc_fastchol_workspace")
    ws = _workspace(size.value, dev)
    tau = torch.empty(graph.n, dtype=torch.float64, device=dev)
    check(L.rwc_fastchol(ctypes.byref(graph.csr), ctypes.byref(p), _ptr(tau), _ptr(ws), ws.numel(), _stream()),
          "rwc_fastchol")
    res = {"tau": tau, "workspace": ws}
    if sync:
        check(L.rwc_workspace_status(_ptr(ws), _stream()), "rwc_fastchol (device status)")
        fe, ie = ctypes.c_int64(), ctypes.c_int64()
        check(L.rwc_fastchol_sizes(_ptr(ws), ctypes.byref(fe), ctypes.byref(ie), _stream()), "rwc_fastchol_sizes")
        res["factor_entries"], res["inverse_entries"] = fe.value, ie.value
    return res


def estimate_group(graph: Graph, roots, counts: torch.Tensor, l: int, tol: float = 1e-12, max_iter: int = 0,
                   want_hit: bool = True, stream_ordered: bool = False) -> dict:
    """Group RWC of the root set S and the estimate of H_{S + u} for every u from forests rooted
    at S (rwc_estimate_group).  Returns group_rwc (a 1-element tensor), marginal [n], hit [n]
    (hitting times to S) and the iteration count."""
    L = _lib.lib()
    dev = graph.device
    rt = _roots_tensor(roots, dev)
    size = ctypes.c_size_t()
    check(L.rwc_estimate_group_workspace(ctypes.byref(graph.csr), ctypes.byref(size)), "rwc_estimate_group_workspace")
    ws = _workspace(size.value, dev)
    grp = torch.empty(1, dtype=torch.float64, device=dev)
    marg = torch.empty(graph.n, dtype=torch.float64, device=dev)
    hit = torch.empty(graph.n, dtype=torch.float64, device=dev) if want_hit else None
    sp = SolveParams(tol=tol, max_iter=max_iter, check_every=_lib.RWC_SOLVE_STREAM_ORDERED if stream_ordered else 0)
    iters = ctypes.c_int32()
    check(L.rwc_estimate_group(ctypes.byref(graph.csr), _ptr(rt), rt.numel(), _ptr(counts), int(l),
                               ctypes.byref(sp), _ptr(grp), _ptr(marg), _ptr(hit), ctypes.byref(iters), _ptr(ws),
                               ws.numel(), _stream()), "rwc_estimate_group")
    return {"group_rwc": grp, "marginal": marg, "hit": hit, "iters": iters.value, "workspace": ws}


def dense_g(n: int, targets, gvals, device) -> torch.Tensor:
    """The vector g (float64 [n] on the device) with g[targets] = gvals, zero elsewhere."""
    g = torch.zeros(n, dtype=torch.float64)
    g[torch.as_tensor(np.asarray(targets, dtype=np.int64))] = torch.as_tensor(np.asarray(gvals, dtype=np.float64))
    return g.to(device)


def backward(graph: Graph, g: torch.Tensor, k: int = 0, seed: int = 0, tol: float = 1e-10,
             max_iter: int = 0, max_support: int | None = None, check_every: int = 0) -> dict:
    """Gradient of sum_j g_j RWC_j with respect to the edge weights (rwc_backward).

    g: float64 [n] device tensor (the upstream gradient).  k = 0 solves one column per nonzero
    of g (exact; the workspace is sized for max_support nonzeros, by default the count of g's
    nonzeros, read once); k > 0 uses k Rademacher probes per sign class of g.  check_every: the
    host looks at convergence every that many iterations (0: 16); iterations launched past it
    return at once, so the result does not depend on it.
    Returns grad_w (float64 [m] on the device, input-edge order) and the CG iterations run."""
    L = _lib.lib()
    gt = _dev_tensor(g, torch.float64, graph.device)
    if gt.numel() != graph.n:
        raise ValueError(f"g must have n = {graph.n} entries, not {gt.numel()}")
    if k == 0 and max_support is None:
        max_support = int(torch.count_nonzero(gt))
    bp = BackwardParams(k=k, max_iter=max_iter, seed=seed, tol=tol, check_every=check_every,
                        max_support=max_support if k == 0 else 0)
    size = ctypes.c_size_t()
    check(L.rwc_backward_workspace(ctypes.byref(graph.csr), ctypes.byref(bp), ctypes.byref(size)),
          "rwc_backward_workspace")
    ws = _workspace(size.value, graph.device)
    grad = torch.empty(graph.m, dtype=torch.float64, device=graph.device)
    iters = ctypes.c_int32()
    check(L.rwc_backward(ctypes.byref(graph.csr), _ptr(gt), ctypes.byref(bp), _ptr(grad), ctypes.byref(iters),
                         _ptr(ws), ws.numel(), _stream()), "rwc_backward")
    return {"grad_w": grad, "iters": iters.value}


class RWCFunction(torch.autograd.Function):
    """RWC as a differentiable function of the edge weights.

    forward:  FastWalk estimate (Algorithm 3: l Wilson trees rooted at the pivot, then AppRWC);
    backward: the analytic gradient of the exact RWC (rwc_backward).  The Monte Carlo
    estimator itself is piecewise constant in w, so its own derivative is useless; the
    backward pass differentiates the quantity it estimates.

    apply(w, n, src, dst, l, seed, k=0, probe_seed=0) with w a float32 CUDA tensor [m]."""

    @staticmethod
    def forward(ctx, w, n, src, dst, l, seed, k=0, probe_seed=0):
        g = Graph(n, src, dst, w.detach().to(torch.float32), w.device)
        s = sample_forests(g, l, seed, want_sq=False, want_hash=False)
        rwc = estimate(g, s["counts"], l, want_hit=False)["rwc"]
        ctx.graph, ctx.k, ctx.probe_seed, ctx.wdtype = g, k, probe_seed, w.dtype
        return rwc

    @staticmethod
    def backward(ctx, grad_rwc):
        gr = grad_rwc.detach().to(torch.float64).contiguous()
        # the upstream gradient goes to the library as it is (a device vector); only the exact
        # mode needs its number of nonzeros to size the workspace
        nnz = int(torch.count_nonzero(gr)) if ctx.k == 0 else None
        if nnz == 0:
            gw = torch.zeros(ctx.graph.m, dtype=ctx.wdtype, device=gr.device)
        else:
            res = backward(ctx.graph, gr, k=ctx.k, seed=ctx.probe_seed, max_support=nnz)
            gw = res["grad_w"].to(ctx.wdtype)
        return gw, None, None, None, None, None, None, None


def random_walk_centrality(n: int, src, dst, w=None, l: int = 2000, seed: int = 0,
                           device: str = "cuda") -> torch.Tensor:
    """FastWalk end to end (Algorithm 3): build the CSR, sample l trees rooted at the pivot,
    assemble RWC.  Returns float64 [n] on the device."""
    g = Graph(n, src, dst, w, device)
    s = sample_forests(g, l, seed, want_sq=False, want_hash=False)
    return estimate(g, s["counts"], l, want_hit=False)["rwc"]


def as_uint64(t: torch.Tensor) -> np.ndarray:
    """Host copy of an int64 tensor reinterpreted as the uint64 values the library wrote."""
    return t.detach().cpu().numpy().view(np.uint64)
