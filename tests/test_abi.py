"""The C-ABI library loads, exports every entry point declared in include/rwc.h, and its
host-only paths (workspace queries, argument validation) behave -- no GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(rwc_\w+)\(", txt, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) <= bound


def test_workspace_queries_and_argument_errors():
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    size = ctypes.c_size_t()
    assert lib.rwc_build_csr_workspace(1000, 4000, 0, ctypes.byref(size)) == 0
    small = size.value
    assert lib.rwc_build_csr_workspace(1000, 4000, 1, ctypes.byref(size)) == 0
    assert size.value > small
    pers = ctypes.c_size_t()
    assert lib.rwc_csr_persistent_bytes(1000, 4000, 1, ctypes.byref(pers)) == 0
    assert 0 < pers.value < size.value
    assert lib.rwc_build_csr_workspace(1, 1, 0, ctypes.byref(size)) == -1      # n < 2
    assert lib.rwc_build_csr_workspace(10, 0, 0, ctypes.byref(size)) == -1     # m < 1
    assert lib.rwc_build_csr_workspace(10, 1 << 31, 0, ctypes.byref(size)) == -7
    # null inputs are rejected before any device work
    csr = _lib.RwcCsr()
    assert lib.rwc_build_csr(10, 5, None, None, None, None, 0, ctypes.byref(csr), None) == -1
    buf = ctypes.create_string_buffer(256)
    assert lib.rwc_last_error(buf, 256) > 0
    assert lib.rwc_status_string(-6) == b"graph is not connected"


def test_sample_workspace_scales_with_trees_in_flight():
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, row_ptr=8, col=8, rec=8, bfs_order=8)
    p = _lib.SampleParams(seed=1, sample_begin=0, num_samples=500, root=-1, trees_in_flight=64,
                          flags=_lib.RWC_SAMPLE_NO_LDS_STATE)
    a = ctypes.c_size_t()
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(a)) == 0
    p.trees_in_flight = 128
    b = ctypes.c_size_t()
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(b)) == 0
    assert b.value - a.value >= 64 * 1000 * 8
    # trees in LDS (this graph's fit) need no slots in HBM at all
    p.flags = 0
    c = ctypes.c_size_t()
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(c)) == 0
    assert c.value < 64 * 1000 * 8
    p.walkers_per_tree = 0
    p.num_samples = 0
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(b)) == -1
    # the sample range must lie in [0, 2^32); the check does not overflow for huge values
    for begin, count in (((1 << 32) - 10, 10), ((1 << 32) - 10, 11), (1 << 62, 1 << 62), (1, (1 << 63) - 1)):
        p.sample_begin, p.num_samples, p.trees_in_flight = begin, count, 8
        want = 0 if begin + count <= (1 << 32) else -1
        assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(b)) == want


def test_package_import_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2510_20604_amd import _lib
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))


def test_flag_constants_match_the_header():
    from paper_2510_20604_amd import _lib
    txt = open(os.path.join(ROOT, "include", "rwc.h")).read()
    defs = dict(re.findall(r"#define\s+(RWC_SAMPLE_\w+)\s+(\d+)u", txt))
    assert len(defs) >= 8
    for name, val in defs.items():
        assert getattr(_lib, name) == int(val), name


def test_exclusive_schedule_flags_are_rejected():
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, row_ptr=8, col=8, rec=8, bfs_order=8)
    size = ctypes.c_size_t()
    for bad in (_lib.RWC_SAMPLE_SPREAD_STARTS | _lib.RWC_SAMPLE_SHARED_STARTS,
                _lib.RWC_SAMPLE_PATH_RING | _lib.RWC_SAMPLE_NO_PATH_RING,
                _lib.RWC_SAMPLE_BFS_STARTS | _lib.RWC_SAMPLE_ID_STARTS):
        p = _lib.SampleParams(seed=1, num_samples=10, root=-1, flags=bad)
        assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(size)) == -1
    p = _lib.SampleParams(seed=1, num_samples=10, root=-1, flags=_lib.RWC_SAMPLE_SPREAD_STARTS | _lib.RWC_SAMPLE_PATH_RING)
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(size)) == 0


def test_library_shares_torchs_hip_runtime():
    """Importing the package (without importing torch first) must leave one HIP runtime in the
    process: a second copy could not open the GPU that torch's copy holds."""
    import subprocess
    import sys
    code = ("import paper_2510_20604_amd\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_backward_sizes_are_checked_before_planning():
    """The adjoint's workspace is sized from k (2 + 2k solve columns, both sign classes) or,
    in exact mode, from max_support; bad sizes are refused without any device work."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, vol=8000.0, row_ptr=8, col=8, rec=8,
                    bfs_order=8)
    size = ctypes.c_size_t()

    def query(k, support=0):
        bp = _lib.BackwardParams(k=k, seed=1, max_support=support)
        return lib.rwc_backward_workspace(ctypes.byref(g), ctypes.byref(bp), ctypes.byref(size))

    assert query(64) == 0
    cols64 = 2 + 2 * 64                       # room for both sign classes
    assert size.value >= 1000 * cols64 * (8 * 3 + 4)
    assert query(0, 3) == 0                   # exact: one column per nonzero of g
    exact3 = size.value
    assert exact3 >= 1000 * 5 * (8 * 3 + 4) and exact3 < 1000 * cols64 * (8 * 3 + 4)
    assert query(0, 0) == -1                  # exact mode needs max_support >= 1
    assert query(0, 1001) == -1               # ... and at most n
    assert query(1 << 23) == -7               # 2 + 2^24 columns
    assert query(-1) == -1


def test_backward_refuses_bad_sizes_before_device_work():
    """rwc_backward checks its parameters before any device call, so a negative or oversized k
    comes back as an error without touching the (dummy) device pointers."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, vol=8000.0, row_ptr=8, col=8, rec=8,
                    bfs_order=8)
    it = ctypes.c_int32()
    for k, support, code in ((-1, 0, -1), (1 << 23, 0, -7), (0, 0, -1), (0, 5000, -1)):
        bp = _lib.BackwardParams(k=k, seed=1, max_support=support)
        assert lib.rwc_backward(ctypes.byref(g), 8, ctypes.byref(bp), 8, ctypes.byref(it), 8, 1 << 20, None) == code
    assert lib.rwc_backward(ctypes.byref(g), None, ctypes.byref(bp), 8, ctypes.byref(it), 8, 1 << 20, None) == -1


def test_sampler_rejects_bad_root_sets_before_device_work():
    """A root set needs a single graph, root = -1, a device pointer and 1 <= count < n."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, row_ptr=8, col=8, rec=8, bfs_order=8)
    size = ctypes.c_size_t()
    ok = _lib.SampleParams(seed=1, num_samples=10, root=-1, roots=8, num_roots=3)
    assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(ok), ctypes.byref(size)) == 0
    for bad in (dict(roots=None, num_roots=3), dict(roots=8, num_roots=-1), dict(roots=8, num_roots=1000),
                dict(roots=8, num_roots=3, root=5)):
        p = _lib.SampleParams(seed=1, num_samples=10, root=bad.get("root", -1), roots=bad["roots"],
                              num_roots=bad["num_roots"])
        assert lib.rwc_sample_forests_workspace(ctypes.byref(g), 1, ctypes.byref(p), ctypes.byref(size)) == -1
    two = (_lib.RwcCsr * 2)(g, g)
    assert lib.rwc_sample_forests_workspace(two, 2, ctypes.byref(ok), ctypes.byref(size)) == -1


def test_estimate_rejects_bad_modes_before_device_work():
    """Stream-ordered solves need 1 <= max_iter <= 4096; the group estimate needs a root count
    in [1, n - 1]."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    g = _lib.RwcCsr(n=1000, pivot=0, m=4000, nnz=8000, weighted=0, vol=8000.0, row_ptr=8, col=8, rec=8,
                    bfs_order=8, strength=8)
    size = ctypes.c_size_t()
    assert lib.rwc_estimate_group_workspace(ctypes.byref(g), ctypes.byref(size)) == 0
    it = ctypes.c_int32()
    for n_roots in (0, 1000):
        assert lib.rwc_estimate_group(ctypes.byref(g), 8, n_roots, 8, 10, None, 8, 8, None, ctypes.byref(it), 8,
                                      size.value, None) == -1
    assert lib.rwc_workspace_status(None, None) == -1
    ws = ctypes.c_size_t()
    assert lib.rwc_estimate_workspace(ctypes.byref(g), ctypes.byref(ws)) == 0
    for max_iter in (0, 5000):
        sp = _lib.SolveParams(tol=1e-12, max_iter=max_iter, check_every=_lib.RWC_SOLVE_STREAM_ORDERED)
        assert lib.rwc_estimate(ctypes.byref(g), 8, None, 10, ctypes.byref(sp), 8, None, None, ctypes.byref(it), 256,
                                ws.value, None) == -1
        assert lib.rwc_estimate_group(ctypes.byref(g), 8, 3, 8, 10, ctypes.byref(sp), 8, 8, None, ctypes.byref(it),
                                      256, size.value, None) == -1


def test_fastchol_method_and_dense_workspace():
    """rwc_fastchol_params.method: AUTO takes the dense form while the (n-1) n / 2 doubles of the
    packed lower triangle fit 32 GiB,
    DENSE holds that array, three per-column words (norm, kept value, its column) and the
    staging area of two columns (16 parts of ceil((n-2)/16) + 1 entries each, with counts,
    pivots and flags) where CHAIN holds its row lists (first and last entry per row, next entry
    and column end per factor entry), and an unknown method or a dense request past 2^20
    columns is refused before any device work."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    assert (_lib.RWC_FASTCHOL_AUTO, _lib.RWC_FASTCHOL_CHAIN, _lib.RWC_FASTCHOL_DENSE) == (0, 1, 2)
    hdr = open(os.path.join(ROOT, "include", "rwc.h")).read()
    for name, val in (("AUTO", 0), ("CHAIN", 1), ("DENSE", 2)):
        assert re.search(rf"#define RWC_FASTCHOL_{name} {val}\b", hdr)

    def ws(n, method):
        g = _lib.RwcCsr(n=n, pivot=0, m=4 * n, nnz=8 * n, weighted=0, row_ptr=8, col=8, rec=8, node_id=8,
                        node_index=8, strength=8)
        p = _lib.FastcholParams(droptol=1e-4, window=16.0, eps_p=1e-3, zeta=16, method=method,
                                factor_capacity=64 * n, inverse_capacity=64 * n)
        size = ctypes.c_size_t()
        rc = lib.rwc_fastchol_workspace(ctypes.byref(g), ctypes.byref(p), ctypes.byref(size))
        return rc, size.value

    rc, chain = ws(1001, _lib.RWC_FASTCHOL_CHAIN)
    assert rc == 0
    rc, dense = ws(1001, _lib.RWC_FASTCHOL_DENSE)
    assert rc == 0
    N, r_cap, cap = 1000, 64 * 1001, -(-999 // 16) + 1
    dense_only = N * (N + 1) // 2 * 8 + N * (8 + 8 + 4) + 2 * 16 * cap * (4 + 8) + 2 * 16 * 4 + 2 * 8 + 2 * 4
    chain_only = N * (8 + 8) + r_cap * (8 + 8)
    assert abs((dense - chain) - (dense_only - chain_only)) <= 13 * 256
    assert ws(1001, _lib.RWC_FASTCHOL_AUTO) == (0, dense)
    big = 92683   # the packed triangle just past 32 GiB: AUTO takes the chain
    assert ws(big, _lib.RWC_FASTCHOL_AUTO) == ws(big, _lib.RWC_FASTCHOL_CHAIN)
    edge = 92682  # just within 32 GiB: still dense
    assert ws(edge, _lib.RWC_FASTCHOL_AUTO) == ws(edge, _lib.RWC_FASTCHOL_DENSE)
    assert ws(1001, 3)[0] == -1
    assert ws(1001, -1)[0] == -1
    assert ws((1 << 20) + 2, _lib.RWC_FASTCHOL_DENSE)[0] == -7


def test_build_flags_are_checked_before_device_work():
    """rwc_build_csr_ex: RWC_BUILD_ALLOW_DISCONNECTED matches the header; unknown bits and null
    inputs are refused before any device call; the CSR's `components` and `component` fields
    sit where the header puts them."""
    from paper_2510_20604_amd import _lib
    lib = _lib.load()
    hdr = open(os.path.join(ROOT, "include", "rwc.h")).read()
    assert re.search(rf"#define RWC_BUILD_ALLOW_DISCONNECTED {_lib.RWC_BUILD_ALLOW_DISCONNECTED}u\b", hdr)
    csr = _lib.RwcCsr()
    assert lib.rwc_build_csr_ex(10, 5, 8, 8, None, 2, 256, 1 << 20, ctypes.byref(csr), None) == -1
    assert lib.rwc_build_csr_ex(10, 5, None, None, None, 1, None, 0, ctypes.byref(csr), None) == -1
    names = [f[0] for f in _lib.RwcCsr._fields_]
    assert names.index("components") == names.index("bfs_depth") + 1
    assert names[-1] == "component"
