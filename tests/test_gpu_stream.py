"""Stream-ordered calls, the status query, the library's cached hipGraph replays and a caller's
own hipGraph capture of sampling plus estimate.

Every replay is checked against the eager result (forest checksums and visit totals bit for
bit, RWC bit for bit), with the program's own eager work and synchronisations between replays.
"""
import numpy as np
import pytest
import torch

import rwcgen as G
from oracle import wilson as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _graph():
    g = G.barabasi_albert(3000, 3, 5)
    return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 6))


def _u64(t):
    return P.as_uint64(t)


def test_sampling_is_stream_ordered_and_reports_status():
    g = _graph()
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.fastwalk_sample(o, o.pivot, 2001, 0, 0, 120)
    s = P.sample_forests(Gd, 120, 2001, sync=False)
    # the call returned without waiting; the status query waits and reports success
    P.workspace_status(s["workspace"])
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])
    # a device-side failure (one walker per tree with a step guard far below what a tree
    # needs, so every walk stops early and exits normally) is reported by the status query,
    # not by the call
    t = P.sample_forests(Gd, 16, 2001, max_steps_per_tree=5, walkers_per_tree=1, sync=False)
    with pytest.raises(P.RWCError) as ei:
        P.workspace_status(t["workspace"])
    assert ei.value.status == -9
    # the next good call on the same workspace clears it
    u = P.sample_forests(Gd, 120, 2001, workspace=t["workspace"], sync=False)
    P.workspace_status(u["workspace"])
    np.testing.assert_array_equal(_u64(u["counts"]), ref["visits"])


def test_library_capture_is_replayed():
    """RWC_SAMPLE_GRAPH_CAPTURE: the first call with a given set of arguments captures, later
    identical calls replay the cached graph; another seed captures anew; all bit-exact."""
    g = _graph()
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    refs = {sd: W.fastwalk_sample(o, o.pivot, sd, 0, 0, 100) for sd in (11, 12)}
    P.release_cached_graphs()
    s = P.sample_forests(Gd, 100, 11, capture=True, persistent=True)
    assert s["graph_replayed"] == 0
    ws = s["workspace"]
    for rep in range(3):
        junk = torch.randn(4096, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        s2 = P.sample_forests(Gd, 100, 11, capture=True, persistent=True, workspace=ws, out=s)
        assert s2["graph_replayed"] == 1, rep
        np.testing.assert_array_equal(_u64(s2["counts"]), refs[11]["visits"])
        np.testing.assert_array_equal(_u64(s2["tree_hash"][0]), refs[11]["hash"])
        del junk
    s3 = P.sample_forests(Gd, 100, 12, capture=True, persistent=True, workspace=ws, out=s)
    assert s3["graph_replayed"] == 0
    np.testing.assert_array_equal(_u64(s3["counts"]), refs[12]["visits"])
    s4 = P.sample_forests(Gd, 100, 11, capture=True, persistent=True, workspace=ws, out=s)
    assert s4["graph_replayed"] == 1
    np.testing.assert_array_equal(_u64(s4["counts"]), refs[11]["visits"])
    P.release_cached_graphs()


def test_stream_ordered_estimate_equals_host_checked():
    """The device-stopped solve runs exactly the iterations of the host-checked one, so the
    outputs are identical bit for bit; the iteration count is read from the workspace."""
    g = _graph()
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, 200, 2001)
    a = P.estimate(Gd, s["counts"], 200, counts_sq=s["counts_sq"], want_stderr=True)
    b = P.estimate(Gd, s["counts"], 200, counts_sq=s["counts_sq"], want_stderr=True, stream_ordered=True,
                   max_iter=2000)
    assert b["iters"] == -1
    P.workspace_status(b["workspace"])
    import ctypes
    it = ctypes.c_int32()
    P._lib.check(P._lib.lib().rwc_workspace_iterations(ctypes.c_void_p(b["workspace"].data_ptr()),
                                                        ctypes.byref(it), ctypes.c_void_p(
                                                            torch.cuda.current_stream().cuda_stream)), "iters")
    assert it.value == a["iters"] > 0
    for key in ("rwc", "hit", "stderr"):
        assert torch.equal(a[key], b[key]), key
    # too few iterations: reported by the status query
    c = P.estimate(Gd, s["counts"], 200, stream_ordered=True, max_iter=3)
    with pytest.raises(P.RWCError) as ei:
        P.workspace_status(c["workspace"])
    assert ei.value.status == -11


def test_caller_captures_sampling_and_estimate():
    """A caller's own hipGraph (torch.cuda.graph) holds one sampling call and one stream-ordered
    estimate; three replays, with other eager work between them, reproduce the eager outputs
    bit for bit."""
    g = _graph()
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    l, seed = 150, 2001
    eager = P.sample_forests(Gd, l, seed)
    eager_est = P.estimate(Gd, eager["counts"], l, stream_ordered=True, max_iter=1000)
    P.workspace_status(eager_est["workspace"])
    prep = P.prepare_sampling(Gd, l, seed=seed)
    # outputs and workspaces allocated before the capture
    s_out = {"counts": torch.empty(g.n, dtype=torch.int64, device="cuda"),
             "counts_sq": torch.empty(g.n, dtype=torch.int64, device="cuda"),
             "total_steps": torch.empty(1, dtype=torch.int64, device="cuda"),
             "tree_hash": torch.empty((1, l), dtype=torch.int64, device="cuda")}
    e_out = {"rwc": torch.empty(g.n, dtype=torch.float64, device="cuda"), "hit": None, "stderr": None}
    e_ws = torch.empty_like(eager_est["workspace"])
    for t in s_out.values():
        t.fill_(-1)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, capture_error_mode="thread_local"):
        s = P.sample_forests(Gd, l, seed, workspace=prep["workspace"], out=s_out, sync=False)
        e = P.estimate(Gd, s["counts"], l, want_hit=False, stream_ordered=True, max_iter=1000, workspace=e_ws,
                       out=e_out)
    torch.cuda.synchronize()
    for rep in range(3):
        s_out["counts"].fill_(0)
        e_out["rwc"].fill_(0.0)
        junk = (torch.arange(1 << 16, device="cuda", dtype=torch.float64) ** 2).sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        P.workspace_status(prep["workspace"])
        P.workspace_status(e_ws)
        assert torch.equal(s_out["counts"], eager["counts"]), rep
        assert torch.equal(s_out["tree_hash"], eager["tree_hash"]), rep
        assert torch.equal(e_out["rwc"], eager_est["rwc"]), rep
        del junk
    del graph


def test_backward_takes_a_device_vector():
    """g goes in as a device vector: zero everywhere gives a zero gradient, a value that is not
    finite or (exact mode) more nonzeros than max_support is refused."""
    g = _graph()
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    assert torch.count_nonzero(P.backward(Gd, z, k=8)["grad_w"]) == 0
    bad = z.clone()
    bad[5] = float("nan")
    with pytest.raises(P.RWCError):
        P.backward(Gd, bad, k=8)
    three = z.clone()
    three[[1, 2, 3]] = 1.0
    with pytest.raises(P.RWCError):
        P.backward(Gd, three, k=0, max_support=2)
    assert torch.isfinite(P.backward(Gd, three, k=0, max_support=3)["grad_w"]).all()
