"""ctypes view of librwc.so (the C ABI declared in include/rwc.h).

Argument marshalling only: every step of the computation runs in the HIP library.  If the
library has not been built this module raises on import; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librwc.so")

c_i32, c_i64, c_u32, c_u64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                                 ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p,
                                                 ctypes.c_size_t)

RWC_BUILD_ALLOW_DISCONNECTED = 1

RWC_SAMPLE_ACCUMULATE = 1
RWC_SAMPLE_PERSISTENT = 2
RWC_SAMPLE_GRAPH_CAPTURE = 4
RWC_SAMPLE_BFS_STARTS = 8
RWC_SAMPLE_SPREAD_STARTS = 16
RWC_SAMPLE_SHARED_STARTS = 32
RWC_SAMPLE_PATH_RING = 64
RWC_SAMPLE_NO_PATH_RING = 128
RWC_SAMPLE_ID_STARTS = 256
RWC_SAMPLE_NO_LDS_STATE = 512

RWC_FASTCHOL_AUTO = 0   # rwc_fastchol_params.method
RWC_FASTCHOL_CHAIN = 1
RWC_FASTCHOL_DENSE = 2

RWC_SOLVE_STREAM_ORDERED = -1   # rwc_solve_params.check_every value selecting stream-ordered mode

STATUS = {
    0: "RWC_OK", -1: "RWC_ERR_INVALID_ARG", -2: "RWC_ERR_NODE_RANGE", -3: "RWC_ERR_SELF_LOOP",
    -4: "RWC_ERR_DUP_EDGE", -5: "RWC_ERR_WEIGHT_RANGE", -6: "RWC_ERR_DISCONNECTED",
    -7: "RWC_ERR_TOO_LARGE", -8: "RWC_ERR_WORKSPACE", -9: "RWC_ERR_STEP_LIMIT",
    -10: "RWC_ERR_COUNT_OVERFLOW", -11: "RWC_ERR_NOT_CONVERGED", -12: "RWC_ERR_HIP", -13: "RWC_ERR_BREAKDOWN",
}


class RwcCsr(ctypes.Structure):
    _fields_ = [("n", c_i32), ("pivot", c_i32), ("m", c_i64), ("nnz", c_i64), ("weighted", c_i32),
                ("max_degree", c_i32), ("vol", c_dbl), ("vol_fixed", c_u64), ("row_ptr", c_vp),
                ("col", c_vp), ("weight", c_vp), ("edge_id", c_vp), ("cdf", c_vp), ("strength", c_vp),
                ("rec", c_vp), ("bfs_order", c_vp), ("bfs_depth", c_i32),
                ("components", c_i32), ("node_id", c_vp), ("node_index", c_vp), ("pivot_index", c_i32),
                ("internal_order", c_i32), ("component", c_vp)]


class SampleParams(ctypes.Structure):
    _fields_ = [("seed", c_u64), ("sample_begin", c_i64), ("num_samples", c_i64), ("root", c_i32),
                ("flags", c_u32), ("trees_in_flight", c_i32), ("walkers_per_tree", c_i32),
                ("max_steps_per_tree", c_u64), ("graph_index_base", c_u32), ("strata", c_u32),
                ("roots", c_vp), ("num_roots", c_i32), ("reserved2", c_i32), ("walkers_per_graph", c_vp)]


class SampleOutputs(ctypes.Structure):
    _fields_ = [("counts", c_vp), ("counts_sq", c_vp), ("total_steps", c_vp), ("tree_hash", c_vp),
                ("parents", c_vp), ("dump_samples", c_vp), ("ndump", c_i32), ("reserved", c_i32),
                ("timing_ms", c_vp), ("plan", c_vp)]


class TrapParams(ctypes.Structure):
    _fields_ = [("seed", c_u64), ("walk_begin", c_i64), ("num_walks", c_i64), ("trap", c_i32),
                ("graph_index", c_u32), ("max_steps_per_walk", c_u64)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("max_iter", c_i32), ("check_every", c_i32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("walkers_per_tree", c_i32), ("trees_in_flight", c_i32), ("steps_per_s", c_dbl),
                ("candidates", c_i32), ("cached", c_i32), ("flags", c_u32), ("reserved", c_i32)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("walkers_mesh", c_i32), ("walkers_other", c_i32), ("flags", c_u32), ("candidates", c_i32),
                ("steps_per_s", c_dbl), ("probe_samples", c_i32), ("cached", c_i32)]


class BackwardParams(ctypes.Structure):
    _fields_ = [("k", c_i32), ("max_iter", c_i32), ("seed", c_u64), ("tol", c_dbl), ("check_every", c_i32),
                ("max_support", c_i32)]


class FastcholParams(ctypes.Structure):
    _fields_ = [("droptol", c_dbl), ("window", c_dbl), ("eps_p", c_dbl), ("zeta", c_i32), ("method", c_i32),
                ("factor_capacity", c_i64), ("inverse_capacity", c_i64)]


# (name, restype, argtypes) for every entry point declared in include/*.h
SIGNATURES = [
    ("rwc_build_csr_workspace", c_i32, [c_i32, c_i64, c_i32, ctypes.POINTER(c_sz)]),
    ("rwc_csr_persistent_bytes", c_i32, [c_i32, c_i64, c_i32, ctypes.POINTER(c_sz)]),
    ("rwc_build_csr", c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_vp, c_sz, ctypes.POINTER(RwcCsr), c_vp]),
    ("rwc_build_csr_ex", c_i32, [c_i32, c_i64, c_vp, c_vp, c_vp, c_u32, c_vp, c_sz, ctypes.POINTER(RwcCsr), c_vp]),
    ("rwc_sample_forests_workspace", c_i32, [ctypes.POINTER(RwcCsr), c_i32, ctypes.POINTER(SampleParams),
                                             ctypes.POINTER(c_sz)]),
    ("rwc_sample_forests", c_i32, [ctypes.POINTER(RwcCsr), c_i32, ctypes.POINTER(SampleParams),
                                   ctypes.POINTER(SampleOutputs), c_vp, c_sz, c_vp]),
    ("rwc_sample_prepare", c_i32, [ctypes.POINTER(RwcCsr), c_i32, ctypes.POINTER(SampleParams), c_vp, c_sz, c_vp]),
    ("rwc_release_cached_graphs", None, []),
    ("rwc_workspace_status", c_i32, [c_vp, c_vp]),
    ("rwc_workspace_iterations", c_i32, [c_vp, ctypes.POINTER(c_i32), c_vp]),
    ("rwc_sample_trap_walks_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(TrapParams),
                                                ctypes.POINTER(c_sz)]),
    ("rwc_sample_trap_walks", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(TrapParams), c_vp, c_vp, c_vp, c_vp,
                                      c_sz, c_vp]),
    ("rwc_estimate_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(c_sz)]),
    ("rwc_estimate", c_i32, [ctypes.POINTER(RwcCsr), c_vp, c_vp, c_i64, ctypes.POINTER(SolveParams), c_vp, c_vp,
                             c_vp, ctypes.POINTER(c_i32), c_vp, c_sz, c_vp]),
    ("rwc_estimate_static", c_i32, [ctypes.POINTER(RwcCsr), c_vp, c_vp, c_i64, ctypes.POINTER(SolveParams), c_vp,
                                    c_vp, c_vp, ctypes.POINTER(c_i32), c_vp]),
    ("rwc_estimate_group_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(c_sz)]),
    ("rwc_estimate_group", c_i32, [ctypes.POINTER(RwcCsr), c_vp, c_i32, c_vp, c_i64, ctypes.POINTER(SolveParams),
                                   c_vp, c_vp, c_vp, ctypes.POINTER(c_i32), c_vp, c_sz, c_vp]),
    ("rwc_estimate_diag", c_i32, [ctypes.POINTER(RwcCsr), c_vp, ctypes.POINTER(SolveParams), c_vp, c_vp,
                                  ctypes.POINTER(c_i32), c_vp, c_sz, c_vp]),
    ("rwc_fastchol_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(FastcholParams), ctypes.POINTER(c_sz)]),
    ("rwc_fastchol", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(FastcholParams), c_vp, c_vp, c_sz, c_vp]),
    ("rwc_fastchol_sizes", c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_vp]),
    ("rwc_backward_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(BackwardParams), ctypes.POINTER(c_sz)]),
    ("rwc_backward", c_i32, [ctypes.POINTER(RwcCsr), c_vp, ctypes.POINTER(BackwardParams), c_vp,
                             ctypes.POINTER(c_i32), c_vp, c_sz, c_vp]),
    ("rwc_autotune_workspace", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(SampleParams), c_i64,
                                       ctypes.POINTER(c_sz)]),
    ("rwc_autotune_sampler", c_i32, [ctypes.POINTER(RwcCsr), ctypes.POINTER(SampleParams), c_i64,
                                     ctypes.POINTER(TuneResult), c_vp, c_sz, c_vp]),
    ("rwc_autotune_batch_workspace", c_i32, [ctypes.POINTER(RwcCsr), c_i32, ctypes.POINTER(SampleParams),
                                             ctypes.POINTER(c_sz)]),
    ("rwc_autotune_batch", c_i32, [ctypes.POINTER(RwcCsr), c_i32, ctypes.POINTER(SampleParams),
                                   ctypes.POINTER(BatchTuneResult), c_vp, c_sz, c_vp]),
    ("rwc_autotune_clear_cache", None, []),
    ("rwc_status_string", ctypes.c_char_p, [c_i32]),
    ("rwc_probe_random_gather", c_i32, [c_vp, c_u64, c_i64, c_i32, c_u32, c_vp, ctypes.POINTER(ctypes.c_float), c_vp]),
    ("rwc_probe_copy", c_i32, [c_vp, c_vp, c_u64, ctypes.POINTER(ctypes.c_float), c_vp]),
    ("rwc_last_error", c_i32, [ctypes.c_char_p, c_sz]),
]


class RWCError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({detail})")


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python paper_2510_20604_amd/build.py)")
    # PyTorch ships its own HIP runtime and loads it by path.  Importing torch first makes
    # librwc.so bind to that same runtime (by soname); loaded the other way round, the process
    # would hold two HIP runtimes and only one of them could open the GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def check(rc: int, where: str) -> None:
    if rc != 0:
        buf = ctypes.create_string_buffer(512)
        lib().rwc_last_error(buf, 512)
        raise RWCError(rc, where, buf.value.decode(errors="replace"))
