"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer outputs (CSR, visit totals, squared visits, step totals, tree checksums, parent
arrays) must be bit-identical.  Floating-point outputs follow tolerances derived in the tests.
"""
import numpy as np
import pytest
import torch

import rwcgen as G
from oracle import exact as E
from oracle import wilson as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _case(name):
    if name == "er1000":
        return G.erdos_renyi_lcc(1000, 8, 1001)
    if name == "er1000_w":
        g = G.erdos_renyi_lcc(1000, 8, 1001)
        return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 3))
    if name == "ba3000":
        return G.barabasi_albert(3000, 3, 5)
    if name == "ba3000_w":
        g = G.barabasi_albert(3000, 3, 5)
        return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 6))
    if name == "grid_w":
        g = G.grid_with_deletions(2500, 0.1, 7)
        return g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, 8))
    if name == "star":
        return G.star_graph(65)
    if name == "path":
        return G.path_graph(130)
    if name == "k2":
        return G.complete_graph(2)
    raise KeyError(name)


CASES = ["er1000", "er1000_w", "ba3000", "ba3000_w", "grid_w", "star", "path", "k2"]


def _u64(t):
    return P.as_uint64(t)


@pytest.mark.parametrize("name", CASES)
def test_csr_matches_oracle(name):
    """The device CSR in its internal order against the oracle's CSR in input order: the order
    (descending weighted degree, ties by id, on heavy-tailed graphs; else the identity), every
    row mapped through it, the records, the start order and the edge ids."""
    g = _case(name)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    nid = Gd.node_id().cpu().numpy()
    nix = Gd.node_index().cpu().numpy()
    np.testing.assert_array_equal(np.sort(nid), np.arange(g.n))
    np.testing.assert_array_equal(nix[nid], np.arange(g.n))
    deg_in = np.diff(o.row_ptr)
    heavy = int(deg_in.max()) * g.n > 8 * g.m
    assert Gd.internal_order == int(heavy)
    if heavy:
        want = np.lexsort((np.arange(g.n), -o.strength))
        np.testing.assert_array_equal(nid, want)
    else:
        np.testing.assert_array_equal(nid, np.arange(g.n))
    assert Gd.pivot == o.pivot
    assert int(Gd.csr.pivot_index) == int(nix[o.pivot])
    assert Gd.vol == o.vol
    deg = deg_in[nid]
    row_ptr = Gd.row_ptr().cpu().numpy()
    np.testing.assert_array_equal(row_ptr, np.concatenate([[0], np.cumsum(deg)]))
    col = Gd.col().cpu().numpy()
    # internal row x holds input node nid[x]'s row, neighbours by ascending input id
    perm = np.concatenate([np.arange(o.row_ptr[p], o.row_ptr[p + 1]) for p in nid]) if g.n else np.zeros(0, int)
    np.testing.assert_array_equal(nid[col], o.col[perm])
    np.testing.assert_array_equal(Gd.strength().cpu().numpy(), o.strength[nid])
    if g.w is not None:
        np.testing.assert_array_equal(_u64(Gd.cdf()), o.cdf[perm])
        np.testing.assert_array_equal(Gd.weight().cpu().numpy().astype(np.float64), o.weight[perm])
    # 64-byte node records: degree, row offset, input id, inline neighbours (and CDF values with
    # the row's total); unused words are zero
    rec = Gd.rec().cpu().numpy().reshape(g.n, 16).view(np.uint32)
    np.testing.assert_array_equal(rec[:, 0], deg)
    np.testing.assert_array_equal(rec[:, 1], row_ptr[:-1])
    np.testing.assert_array_equal(rec[:, 2], nid)
    inline = 3 if g.w is not None else 13
    lo32 = np.uint64(0xFFFFFFFF)
    cdf = _u64(Gd.cdf()) if g.w is not None else None
    for x in range(0, g.n, max(1, g.n // 200)):
        b, k = row_ptr[x], min(deg[x], inline)
        want = np.zeros(16, dtype=np.uint32)
        want[0], want[1], want[2] = deg[x], b, nid[x]
        want[3:3 + k] = col[b:b + k]
        if g.w is not None:
            c = cdf[b:b + k].astype(np.uint64)
            want[8:8 + 2 * k:2] = (c & lo32).astype(np.uint32)
            want[9:9 + 2 * k:2] = (c >> np.uint64(32)).astype(np.uint32)
            total = np.uint64(cdf[row_ptr[x + 1] - 1])
            want[6], want[7] = np.uint32(total & lo32), np.uint32(total >> np.uint64(32))
        np.testing.assert_array_equal(rec[x], want, err_msg=f"record of internal node {x}")
    # breadth-first start order (internal indices): a permutation starting at the pivot,
    # distances non-decreasing
    order = Gd.bfs_order().cpu().numpy()
    np.testing.assert_array_equal(np.sort(order), np.arange(g.n))
    assert order[0] == nix[o.pivot]
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    A = sp.csr_matrix((np.ones(o.col.shape[0]), o.col, o.row_ptr), shape=(g.n, g.n))
    dist = csg.shortest_path(A, unweighted=True, indices=o.pivot)
    assert np.all(np.diff(dist[nid[order]]) >= 0)
    assert Gd.csr.bfs_depth == int(dist.max())        # the pivot's eccentricity
    # edge_id maps every entry back to an input edge with matching endpoints
    eid = Gd.edge_id().cpu().numpy()
    rows = np.repeat(nid, deg)
    a, b = g.src[eid], g.dst[eid]
    assert np.all(((a == rows) & (b == nid[col])) | ((b == rows) & (a == nid[col])))


@pytest.mark.parametrize("bad,code", [("self_loop", -3), ("dup", -4), ("range", -2), ("weight", -5),
                                      ("disconnected", -6), ("nan", -5)])
def test_csr_rejects_bad_input(bad, code):
    src = np.array([0, 1, 2, 3], dtype=np.int32)
    dst = np.array([1, 2, 3, 0], dtype=np.int32)
    w = None
    n = 4
    if bad == "self_loop":
        dst[1] = 1
    elif bad == "dup":
        src[3], dst[3] = 1, 0
    elif bad == "range":
        dst[2] = 7
    elif bad == "weight":
        w = np.array([1.0, 0.25, 1.0, 1.0], dtype=np.float32)
    elif bad == "nan":
        w = np.array([1.0, np.nan, 1.0, 1.0], dtype=np.float32)
    elif bad == "disconnected":
        n = 6
    with pytest.raises(P.RWCError) as ei:
        P.Graph(n, src, dst, w)
    assert ei.value.status == code


@pytest.fixture(scope="module")
def oracle_runs():
    cache = {}

    def get(name, l, seed, graph=0, sample_begin=0):
        key = (name, l, seed, graph, sample_begin)
        if key not in cache:
            g = _case(name)
            o = W.OracleCSR(g.n, g.src, g.dst, g.w)
            cache[key] = (g, o, W.fastwalk_sample(o, o.pivot, seed, graph, sample_begin, l,
                                                  want_parents=True, threads=8))
        return cache[key]

    return get


@pytest.mark.parametrize("name,l", [("er1000", 2000), ("er1000_w", 300), ("ba3000", 200), ("ba3000_w", 200),
                                    ("grid_w", 100), ("star", 50), ("path", 70), ("k2", 10)])
@pytest.mark.parametrize("lds", [None, False])
def test_forest_bit_exact(name, l, lds, oracle_runs):
    """The automatic plan (small graphs: trees in LDS) and tree state in HBM slots."""
    g, o, ref = oracle_runs(name, l, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    dump = list(range(min(16, l)))
    s = P.sample_forests(Gd, l, 2001, dump=dump, lds_state=lds)
    assert (s["lds_graphs"] == 1) == (lds is None and s["walkers_per_tree"] > 1)
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["counts_sq"]), ref["visits_sq"])
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(s["parents"].cpu().numpy(), ref["parents"][dump])
    assert int(_u64(s["total_steps"])[0]) == int(ref["steps"].sum())


@pytest.mark.parametrize("tif,persistent,capture", [(64, False, False), (128, True, False), (192, False, True),
                                                    (64, True, True)])
def test_launch_shape_does_not_change_the_forest(tif, persistent, capture, oracle_runs):
    g, o, ref = oracle_runs("er1000_w", 300, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, 300, 2001, trees_in_flight=tif, persistent=persistent, capture=capture, dump=[0, 299],
                         lds_state=False)
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["counts_sq"]), ref["visits_sq"])
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(s["parents"].cpu().numpy(), ref["parents"][[0, 299]])


@pytest.mark.parametrize("walkers", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("name,l", [("er1000", 150), ("er1000_w", 100), ("ba3000", 70), ("ba3000_w", 70), ("grid_w", 40),
                                    ("star", 20), ("path", 30), ("k2", 8)])
@pytest.mark.parametrize("lds", [None, False])
def test_walker_teams_are_bit_exact(walkers, name, l, lds, oracle_runs):
    """Several walkers per tree pop the same cycles as the serial order of Algorithm 3, with
    the trees' state in LDS (the default for these small graphs) or in HBM."""
    g, o, ref = oracle_runs(name, l, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    dump = [0, l - 1]
    s = P.sample_forests(Gd, l, 2001, walkers_per_tree=walkers, dump=dump, lds_state=lds)
    fits = walkers > 1 and (64 // walkers) * ((g.n + 7) // 8 * 8) * 8 <= 48 * 1024   # 64 / W trees in 48 KB
    assert s["walk_kernel"].startswith("wilson_team_lds") == (fits and lds is None)
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(s["parents"].cpu().numpy(), ref["parents"][dump])
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["counts_sq"]), ref["visits_sq"])
    assert int(_u64(s["total_steps"])[0]) == int(ref["steps"].sum())


@pytest.mark.parametrize("walkers,tif,persistent,bfs,starts,ring", [
    (8, 16, True, False, "shared", False), (16, 4, False, True, "shared", None),
    (64, 3, True, False, "spread", None), (4, 32, False, True, "spread", False),
    (64, 200, False, False, "shared", True), (32, 7, True, True, "auto", True),
    (2, 64, False, False, "spread", True), (64, 64, True, False, "auto", None)])
@pytest.mark.parametrize("name", ["ba3000_w", "grid_w", "path"])
def test_walker_teams_launch_shapes(walkers, tif, persistent, bfs, starts, ring, name, oracle_runs):
    """Start order, start sharing, the LDS path ring and the launch shape only change the
    schedule: the forest and the visit counts stay those of the serial order."""
    g, o, ref = oracle_runs(name, 200, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, 200, 2001, walkers_per_tree=walkers, trees_in_flight=tif, persistent=persistent,
                         lds_state=(False if tif % 2 else None),
                         bfs_starts=bfs, starts=starts, path_ring=ring)
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])


def test_sample_range_chunks_accumulate(oracle_runs):
    g, o, ref = oracle_runs("ba3000_w", 200, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    a = P.sample_forests(Gd, 70, 2001, sample_begin=0)
    b = P.sample_forests(Gd, 130, 2001, sample_begin=70, accumulate={k: a[k] for k in
                                                                    ("counts", "counts_sq", "total_steps")})
    np.testing.assert_array_equal(_u64(b["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(b["counts_sq"]), ref["visits_sq"])
    np.testing.assert_array_equal(_u64(b["tree_hash"][0]), ref["hash"][70:])


def test_batched_graphs_match_per_graph_oracle():
    graphs = G.batch_mix(6, 300, 3000, seed=41)
    dev = [P.Graph(g.n, g.src, g.dst, g.w) for g in graphs]
    l, seed, base = 64 + 17, 77, 5
    s = P.sample_forests(dev, l, seed, persistent=True, capture=True, graph_index_base=base)
    counts = _u64(s["counts"])
    off = 0
    for i, g in enumerate(graphs):
        o = W.OracleCSR(g.n, g.src, g.dst, g.w)
        ref = W.fastwalk_sample(o, o.pivot, seed, base + i, 0, l, threads=8)
        np.testing.assert_array_equal(counts[off:off + g.n], ref["visits"])
        np.testing.assert_array_equal(_u64(s["tree_hash"][i]), ref["hash"])
        off += g.n
    # plain per-graph launches give the same bits
    for i, gd in enumerate(dev[:2]):
        p = P.sample_forests(gd, l, seed, graph_index_base=base + i)
        np.testing.assert_array_equal(_u64(p["tree_hash"][0]), _u64(s["tree_hash"][i]))
    # and so does the batch with one walker per tree (the single-lane kernel, persistent)
    s1 = P.sample_forests(dev, l, seed, persistent=True, graph_index_base=base, walkers_per_tree=1)
    assert s1["walk_kernel"] == "wilson_walk"
    np.testing.assert_array_equal(_u64(s1["counts"]), counts)
    np.testing.assert_array_equal(_u64(s1["tree_hash"]), _u64(s["tree_hash"]))


def test_batched_mixed_team_widths_match_oracle():
    """A batch whose graphs get different walkers per tree (16, 32 and 64 by size) and different
    start modes (shared for BA, spread for the meshes) in one persistent launch reproduces each
    graph's serial forest."""
    gs = [G.barabasi_albert(300, 3, 51), G.grid_with_deletions(9000, 0.1, 52), G.barabasi_albert(20000, 3, 53),
          G.grid_with_deletions(600, 0.1, 54)]
    gs = [g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 60 + i)) for i, g in enumerate(gs)]
    dev = [P.Graph(g.n, g.src, g.dst, g.w) for g in gs]
    l, seed = 40, 91
    s = P.sample_forests(dev, l, seed, persistent=True)
    counts = _u64(s["counts"])
    off = 0
    for i, g in enumerate(gs):
        o = W.OracleCSR(g.n, g.src, g.dst, g.w)
        ref = W.fastwalk_sample(o, o.pivot, seed, i, 0, l, threads=8)
        np.testing.assert_array_equal(counts[off:off + g.n], ref["visits"])
        np.testing.assert_array_equal(_u64(s["tree_hash"][i]), ref["hash"])
        off += g.n
    # and with a forced small number of trees in flight (several batches, all graphs)
    s2 = P.sample_forests(dev, l, seed, persistent=True, trees_in_flight=16)
    np.testing.assert_array_equal(_u64(s2["counts"]), counts)
    np.testing.assert_array_equal(_u64(s2["tree_hash"]), _u64(s["tree_hash"]))


def test_explicit_root(oracle_runs):
    g = _case("er1000_w")
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.fastwalk_sample(o, 17, 5, 0, 0, 40)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, 40, 5, root=17)
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])


def test_step_guard_reports_an_error():
    g = _case("grid_w")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    with pytest.raises(P.RWCError) as ei:
        P.sample_forests(Gd, 8, 1, max_steps_per_tree=100, walkers_per_tree=1)
    assert ei.value.status == -9


# ----------------------------------------------------------------------- estimate -----
@pytest.mark.parametrize("name,l", [("er1000", 2000), ("er1000_w", 300), ("ba3000_w", 200), ("grid_w", 100)])
def test_estimate_matches_oracle_assembly(name, l, oracle_runs):
    """rwc_estimate on the same visit totals reproduces Algorithm 1 evaluated with a dense FP64
    solve.  The CG stops at relative residual 1e-12 of L_v h = d; the error this leaves in h is
    at most cond(L_v) * 1e-12 relative, which the test bounds with cond <= 1e3 for these graphs
    (plus rounding), hence 1e-9."""
    g, o, ref = oracle_runs(name, l, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    counts = torch.as_tensor(ref["visits"].view(np.int64)).cuda()
    counts_sq = torch.as_tensor(ref["visits_sq"].view(np.int64)).cuda()
    est = P.estimate(Gd, counts, l, counts_sq=counts_sq, want_stderr=True)
    want = E.fastwalk_estimate(g.n, g.src, g.dst, g.w, o.pivot, ref["visits"], l)
    got = est["rwc"].cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-9)
    hit = E.hitting_times_to(g.n, g.src, g.dst, g.w, o.pivot)
    np.testing.assert_allclose(est["hit"].cpu().numpy(), hit, rtol=1e-9, atol=1e-9 * hit.max())
    # the estimate is within its own error bars of the exact RWC for most nodes
    exact = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w)
    se = est["stderr"].cpu().numpy()
    mask = se > 0
    z = np.abs(got[mask] - exact[mask]) / se[mask]
    assert np.mean(z > 4) < 0.01


def test_end_to_end_er1000_accuracy():
    g = _case("er1000")
    rwc = P.random_walk_centrality(g.n, g.src, g.dst, None, l=2000, seed=2001).cpu().numpy()
    exact = E.rwc_laplacian_pinv(g.n, g.src, g.dst, None)
    mre = E.mean_relative_error(exact, rwc)
    assert mre < 0.03


def test_autotuner_choice_does_not_change_the_forest(oracle_runs):
    g, o, ref = oracle_runs("ba3000_w", 200, 2001)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    from paper_2510_20604_amd import _lib
    _lib.lib().rwc_autotune_clear_cache()
    t = P.autotune(Gd, 200, 2001)
    assert t["candidates"] >= 2 and not t["cached"]
    assert t["walkers_per_tree"] in (1, 8, 16, 32, 64) and t["trees_in_flight"] >= 1
    if t["walkers_per_tree"] == 1:
        assert t["path_ring"] is None and t["starts"] == "auto" and t["bfs_starts"] is None
    s = P.sample_forests(Gd, 200, 2001, walkers_per_tree=t["walkers_per_tree"],
                         trees_in_flight=t["trees_in_flight"], path_ring=t["path_ring"], starts=t["starts"],
                         bfs_starts=t["bfs_starts"], lds_state=t["lds_state"])
    np.testing.assert_array_equal(_u64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(_u64(s["tree_hash"][0]), ref["hash"])
    again = P.autotune(Gd, 200, 2001)
    assert again["cached"] and again["walkers_per_tree"] == t["walkers_per_tree"]


def test_batch_autotuner_choice_does_not_change_the_forests():
    """rwc_autotune_batch on a mixed batch (BA graphs and meshes): the tuned call (per-class
    walkers, schedule, LDS choice) gives the automatic plan's outputs bit for bit, and both
    match the oracle on two graphs; a second tuning call is served from the cache."""
    graphs = G.batch_mix(8, 500, 8000, seed=47)
    dev = [P.Graph(g.n, g.src, g.dst, g.w) for g in graphs]
    l, seed = 96, 13
    P._lib.lib().rwc_autotune_clear_cache()
    t = P.autotune_batch(dev, l, seed)
    assert t["candidates"] == 17 and not t["cached"]
    assert t["walkers_mesh"] in (16, 32, 64) and t["walkers_other"] in (16, 32, 64)
    assert P.autotune_batch(dev, l, seed)["cached"]
    auto = P.sample_forests(dev, l, seed, persistent=True)
    tuned = P.sample_forests(dev, l, seed, persistent=True, walkers_per_graph=t["walkers_per_graph"],
                             path_ring=t["path_ring"], bfs_starts=t["bfs_starts"], lds_state=t["lds_state"])
    for key in ("counts", "counts_sq", "tree_hash", "total_steps"):
        assert torch.equal(auto[key], tuned[key]), key
    off = 0
    counts = _u64(tuned["counts"])
    for i, g in enumerate(graphs):
        if i in (0, len(graphs) - 1):
            o = W.OracleCSR(g.n, g.src, g.dst, g.w)
            ref = W.fastwalk_sample(o, o.pivot, seed, i, 0, l, threads=8)
            np.testing.assert_array_equal(counts[off:off + g.n], ref["visits"])
            np.testing.assert_array_equal(_u64(tuned["tree_hash"][i]), ref["hash"])
        off += g.n


@pytest.mark.parametrize("shape", ["star", "bipartite"])
def test_csr_rejects_fixed_point_overflow(shape):
    """Weights near the top of the accepted range on long rows: a star whose centre row passes
    2^64 in fixed point (the row carry saturates instead of wrapping), and a complete bipartite
    graph K(2048, 4100) whose rows all stay below 2^53 but whose total passes 2^64 (the volume
    check).  Both are refused with RWC_ERR_WEIGHT_RANGE."""
    if shape == "star":
        leaves = (1 << 24) + (1 << 18)
        src = np.zeros(leaves, dtype=np.int32)
        dst = np.arange(1, leaves + 1, dtype=np.int32)
        n = leaves + 1
    else:
        a, b = 2048, 4100
        src = np.repeat(np.arange(a, dtype=np.int32), b)
        dst = (a + np.tile(np.arange(b, dtype=np.int32), a)).astype(np.int32)
        n = a + b
    w = np.full(src.shape[0], 65535.99609375, dtype=np.float32)    # the largest float32 below 65536
    assert float(w[0]) < 65536.0
    with pytest.raises(P.RWCError) as ei:
        P.Graph(n, src, dst, w)
    assert ei.value.status == -5


def test_breadth_first_order_with_long_frontier_rows():
    """A hub of 5000 leaves, 300 of which are hubs of 4100 leaves each: rows longer than 4096
    entries are shared by every wave of a level, and the second level has more of them (300)
    than one level defers (256), so the rest are expanded in place.  The start order is a
    permutation from the pivot with non-decreasing distance, and the depth is the pivot's
    eccentricity."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    hubs, leaves, sub = 5000, 300, 4100
    src = [np.zeros(hubs, np.int64)]
    dst = [1 + np.arange(hubs)]
    nxt = 1 + hubs
    for h in range(leaves):
        src.append(np.full(sub, 1 + h, np.int64))
        dst.append(nxt + np.arange(sub))
        nxt += sub
    src, dst, n = np.concatenate(src), np.concatenate(dst), nxt
    Gd = P.Graph(n, src, dst)
    order = Gd.bfs_order().cpu().numpy()
    nid = Gd.node_id().cpu().numpy()
    np.testing.assert_array_equal(np.sort(order), np.arange(n))
    assert nid[order[0]] == Gd.pivot
    A = sp.csr_matrix((np.ones(2 * len(src)), (np.concatenate([src, dst]), np.concatenate([dst, src]))),
                      shape=(n, n))
    dist = csg.shortest_path(A, unweighted=True, indices=Gd.pivot)
    assert np.all(np.diff(dist[nid[order]]) >= 0)
    assert Gd.csr.bfs_depth == int(dist.max())
