"""rwc_estimate_static (the estimate over the library's fixed device array, for callers that
cannot allocate) against rwc_estimate with a caller workspace, through the C ABI: identical
outputs on two calls in a row, the second on a smaller graph, and the size and mode limits."""
import ctypes

import numpy as np
import pytest
import torch

import rwcgen as G

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_static_estimate_matches_workspace_estimate_on_two_calls():
    lib = P._lib.lib()
    cases = [(G.barabasi_albert(20_000, 5, 1002), None, 300),
             (G.erdos_renyi_lcc(1000, 8, 1001), 0.5, 200)]   # the second call is smaller
    for g, wlo, l in cases:
        w = None if wlo is None else G.uniform_weights(g.m, wlo, 2.0, 3)
        Gd = P.Graph(g.n, g.src, g.dst, w)
        s = P.sample_forests(Gd, l, 2001)
        ref = P.estimate(Gd, s["counts"], l, counts_sq=s["counts_sq"], want_stderr=True)
        rwc = torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda")
        hit = torch.full_like(rwc, -1.0)
        se = torch.full_like(rwc, -1.0)
        it = ctypes.c_int32()
        sp = P._lib.SolveParams(tol=1e-12, max_iter=0, check_every=0)
        rc = lib.rwc_estimate_static(ctypes.byref(Gd.csr), _vp(s["counts"]), _vp(s["counts_sq"]), l,
                                     ctypes.byref(sp), _vp(rwc), _vp(hit), _vp(se), ctypes.byref(it), _stream())
        assert rc == 0
        assert it.value == ref["iters"] > 0
        assert torch.equal(rwc, ref["rwc"])
        assert torch.equal(hit, ref["hit"])
        assert torch.equal(se, ref["stderr"])


def test_static_estimate_limits():
    """A graph too large for the fixed array and the stream-ordered mode are refused before
    any device work."""
    lib = P._lib.lib()
    g = P._lib.RwcCsr(n=4_000_000, pivot=0, m=8_000_000, nnz=16_000_000, row_ptr=8, col=8, rec=8, bfs_order=8,
                      strength=8, vol=1.6e7)
    it = ctypes.c_int32()
    sp = P._lib.SolveParams(tol=1e-12, max_iter=0, check_every=0)
    assert lib.rwc_estimate_static(ctypes.byref(g), 8, None, 10, ctypes.byref(sp), 8, None, None, ctypes.byref(it),
                                   _stream()) == -7
    g.n = 1000
    sp.check_every = P._lib.RWC_SOLVE_STREAM_ORDERED
    sp.max_iter = 100
    assert lib.rwc_estimate_static(ctypes.byref(g), 8, None, 10, ctypes.byref(sp), 8, None, None, ctypes.byref(it),
                                   _stream()) == -1
