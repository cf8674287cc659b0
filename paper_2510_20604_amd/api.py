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
from ._lib import BackwardParams, RwcCsr, SampleOutputs, SampleParams, SolveParams, TuneResult, check


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
    """An undirected graph built on the device by rwc_build_csr."""

    def __init__(self, n: int, src, dst, w=None, device: str | torch.device = "cuda"):
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
        check(L.rwc_build_csr(self.n, self.m, _ptr(self.src), _ptr(self.dst), _ptr(self.w), _ptr(self.ws),
                              self.ws.numel(), ctypes.byref(self.csr), _stream()), "rwc_build_csr")

    # -- views of the device CSR (for tests and diagnostics) --
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

    def rec(self) -> torch.Tensor:
        return self._view(self.csr.rec, 16 * self.n, torch.int32)


def sample_forests(graphs: Graph | Sequence[Graph], num_samples: int, seed: int, sample_begin: int = 0,
                   root: int = -1, trees_in_flight: int = 0, walkers_per_tree: int = 0,
                   persistent: bool = False, capture: bool = False, want_sq: bool = True,
                   want_hash: bool = True, dump: Sequence[int] = (), max_steps_per_tree: int = 0,
                   graph_index_base: int = 0, accumulate: dict | None = None,
                   workspace: torch.Tensor | None = None, timing: bool = False,
                   bfs_starts: bool | None = None, starts: str = "auto", path_ring: bool | None = None) -> dict:
    """Samples `num_samples` rooted spanning trees of every graph (rwc_sample_forests).

    Returns device tensors: counts [sum n] (int64 holding uint64 values), counts_sq,
    total_steps [G], tree_hash [G, num_samples], parents [len(dump), n] and the workspace
    used (pass it back as `workspace` to reuse it).  With timing=True also walk_ms and
    reduce_ms: device time of the walk and reduction kernels (hipEvents on the stream).
    `starts` ("auto", "shared", "spread"), `bfs_starts` (None = automatic, True =
    breadth-first from the root, False = ascending ids) and `path_ring` (None = automatic) pick
    how walker teams schedule their walks; the forest does not depend on them."""
    L = _lib.lib()
    gl = [graphs] if isinstance(graphs, Graph) else list(graphs)
    G = len(gl)
    dev = gl[0].device
    arr = (RwcCsr * G)(*[g.csr for g in gl])
    flags = 0
    if persistent:
        flags |= _lib.RWC_SAMPLE_PERSISTENT
    if capture:
        flags |= _lib.RWC_SAMPLE_GRAPH_CAPTURE
    if accumulate is not None:
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
    p = SampleParams(seed=seed, sample_begin=sample_begin, num_samples=num_samples, root=root, flags=flags,
                     trees_in_flight=trees_in_flight, walkers_per_tree=walkers_per_tree,
                     max_steps_per_tree=max_steps_per_tree, graph_index_base=graph_index_base)
    size = ctypes.c_size_t()
    check(L.rwc_sample_forests_workspace(arr, G, ctypes.byref(p), ctypes.byref(size)),
          "rwc_sample_forests_workspace")
    if workspace is None or workspace.numel() < size.value:
        workspace = _workspace(size.value, dev)
    total = sum(g.n for g in gl)
    if accumulate is not None:
        res = accumulate
    else:
        res = {
            "counts": torch.empty(total, dtype=torch.int64, device=dev),
            "counts_sq": torch.empty(total, dtype=torch.int64, device=dev) if want_sq else None,
            "total_steps": torch.empty(G, dtype=torch.int64, device=dev),
        }
    res["tree_hash"] = torch.empty((G, num_samples), dtype=torch.int64, device=dev) if want_hash else None
    dump = list(dump)
    res["parents"] = torch.empty((len(dump), gl[0].n), dtype=torch.int32, device=dev) if dump else None
    dump_host = (ctypes.c_int64 * max(1, len(dump)))(*dump) if dump else None
    out = SampleOutputs(counts=_ptr(res["counts"]), counts_sq=_ptr(res.get("counts_sq")),
                        total_steps=_ptr(res.get("total_steps")), tree_hash=_ptr(res["tree_hash"]),
                        parents=_ptr(res["parents"]),
                        dump_samples=ctypes.cast(dump_host, ctypes.c_void_p) if dump else None,
                        ndump=len(dump))
    tms = (ctypes.c_float * 2)()
    if timing:
        out.timing_ms = ctypes.cast(tms, ctypes.c_void_p)
    plan = (ctypes.c_int32 * 6)()
    out.plan = ctypes.cast(plan, ctypes.c_void_p)
    check(L.rwc_sample_forests(arr, G, ctypes.byref(p), ctypes.byref(out), _ptr(workspace), workspace.numel(),
                               _stream()), "rwc_sample_forests")
    res["workspace"] = workspace
    res["walkers_per_tree"], res["trees_in_flight"], res["batches"] = int(plan[0]), int(plan[1]), int(plan[2])
    res["walk_kernel"] = ("wilson_walk", "wilson_team<false>", "wilson_team<true>")[int(plan[3])]
    res["starts"] = "spread" if plan[4] else "shared"
    res["start_order"] = "breadth-first" if plan[5] else "ascending"
    if timing:
        res["walk_ms"], res["reduce_ms"] = float(tms[0]), float(tms[1])
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
            "bfs_starts": pick(_lib.RWC_SAMPLE_BFS_STARTS, _lib.RWC_SAMPLE_ID_STARTS, True, False, None)}


def estimate(graph: Graph, counts: torch.Tensor, l: int, counts_sq: torch.Tensor | None = None,
             tol: float = 1e-12, max_iter: int = 0, want_hit: bool = True, want_stderr: bool = False) -> dict:
    """RWC from visit totals (rwc_estimate): returns rwc, hit (hitting times to the pivot),
    stderr and the CG iteration count."""
    L = _lib.lib()
    dev = graph.device
    size = ctypes.c_size_t()
    check(L.rwc_estimate_workspace(ctypes.byref(graph.csr), ctypes.byref(size)), "rwc_estimate_workspace")
    ws = _workspace(size.value, dev)
    rwc = torch.empty(graph.n, dtype=torch.float64, device=dev)
    hit = torch.empty(graph.n, dtype=torch.float64, device=dev) if want_hit else None
    se = torch.empty(graph.n, dtype=torch.float64, device=dev) if want_stderr else None
    sp = SolveParams(tol=tol, max_iter=max_iter, check_every=0)
    iters = ctypes.c_int32()
    check(L.rwc_estimate(ctypes.byref(graph.csr), _ptr(counts), _ptr(counts_sq), int(l), ctypes.byref(sp),
                         _ptr(rwc), _ptr(hit), _ptr(se), ctypes.byref(iters), _ptr(ws), ws.numel(), _stream()),
          "rwc_estimate")
    return {"rwc": rwc, "hit": hit, "stderr": se, "iters": iters.value}


def backward(graph: Graph, targets, gvals, k: int = 0, seed: int = 0, tol: float = 1e-10,
             max_iter: int = 0) -> dict:
    """Gradient of sum_j g_j RWC_j with respect to the edge weights (rwc_backward).

    targets / gvals: the nodes with nonzero g and their values (host arrays).  k = 0 solves
    one column per target (exact); k > 0 uses k Rademacher probes per sign class of g.
    Returns grad_w (float64 [m] on the device, input-edge order) and the CG iterations."""
    L = _lib.lib()
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    gv = np.ascontiguousarray(np.asarray(gvals, dtype=np.float64))
    if t.shape != gv.shape or t.ndim != 1 or t.size == 0:
        raise ValueError("targets and gvals must be matching non-empty 1-D arrays")
    bp = BackwardParams(k=k, max_iter=max_iter, seed=seed, tol=tol, check_every=0)
    tp = t.ctypes.data_as(ctypes.c_void_p)
    gp = gv.ctypes.data_as(ctypes.c_void_p)
    size = ctypes.c_size_t()
    check(L.rwc_backward_workspace(ctypes.byref(graph.csr), t.size, tp, gp, ctypes.byref(bp), ctypes.byref(size)),
          "rwc_backward_workspace")
    ws = _workspace(size.value, graph.device)
    grad = torch.empty(graph.m, dtype=torch.float64, device=graph.device)
    iters = ctypes.c_int32()
    check(L.rwc_backward(ctypes.byref(graph.csr), t.size, tp, gp, ctypes.byref(bp), _ptr(grad), ctypes.byref(iters),
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
        gr = grad_rwc.detach().to(torch.float64)
        nz = torch.nonzero(gr).flatten()
        if nz.numel() == 0:
            gw = torch.zeros(ctx.graph.m, dtype=ctx.wdtype, device=gr.device)
        else:
            res = backward(ctx.graph, nz.cpu().numpy(), gr[nz].cpu().numpy(), k=ctx.k, seed=ctx.probe_seed)
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
