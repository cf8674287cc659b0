"""Spanning forests rooted at a set S (InTree = S at the start of every sample) and the group
random walk centrality built on them, against the oracle.

Forests (integer outputs) must be bit-identical to the oracle's serial sampler under the same
keys, for one walker per tree and for walker teams.  The group estimate is floating point: the
GPU's and the oracle's assembly of the same visit totals agree to 1e-9 relative (both solve the
system grounded at S to a relative residual of 1e-12, far below that).
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
    if name == "er1000_w":
        g = G.erdos_renyi_lcc(1000, 8, 1001)
        g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 3))
        return g, np.random.default_rng(1).choice(g.n, 5, replace=False)
    if name == "ba3000":
        g = G.barabasi_albert(3000, 3, 5)
        return g, np.random.default_rng(2).choice(g.n, 20, replace=False)
    if name == "grid_w":
        g = G.grid_with_deletions(2500, 0.1, 7)
        g = g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, 8))
        return g, np.array([0, g.n - 1])
    if name == "path":
        g = G.path_graph(130)
        return g, np.array([0, 64, 129])
    raise KeyError(name)


@pytest.mark.parametrize("walkers", [1, 8, 64])
@pytest.mark.parametrize("name,l", [("er1000_w", 200), ("ba3000", 100), ("grid_w", 40), ("path", 50)])
def test_root_set_forests_bit_exact(name, l, walkers):
    g, S = _case(name)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.fastwalk_sample(o, S, 2001, 0, 0, l, want_parents=True, threads=8)
    s = P.sample_forests(Gd, l, 2001, roots=S, walkers_per_tree=walkers, dump=[0, l - 1])
    np.testing.assert_array_equal(P.as_uint64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(P.as_uint64(s["counts_sq"]), ref["visits_sq"])
    np.testing.assert_array_equal(P.as_uint64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(s["parents"].cpu().numpy(), ref["parents"][[0, l - 1]])
    assert int(P.as_uint64(s["total_steps"])[0]) == int(ref["steps"].sum())


def test_root_set_of_one_is_the_rooted_tree():
    g, _ = _case("ba3000")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    a = P.sample_forests(Gd, 64, 7, roots=[Gd.pivot])
    b = P.sample_forests(Gd, 64, 7)
    for key in ("counts", "counts_sq", "tree_hash", "total_steps"):
        assert torch.equal(a[key], b[key]), key


@pytest.mark.parametrize("roots,code", [([3, 9, 3], -1), ([3, 5000], -2), ([-1, 4], -2)])
def test_bad_root_sets_are_reported(roots, code):
    g, _ = _case("ba3000")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    with pytest.raises(P.RWCError) as ei:
        P.sample_forests(Gd, 8, 7, roots=roots)
    assert ei.value.status == code


@pytest.mark.parametrize("name", ["er1000_w", "grid_w"])
def test_group_estimate_matches_oracle_assembly(name):
    """H_S and H_{S + u} for every u from the GPU's visit totals, against the oracle's
    definition-based hitting times and the same rank-one assembly; the stream-ordered solve
    gives the same bits as the host-checked one."""
    g, S = _case(name)
    l = 100
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, l, 2001, roots=S)
    counts = P.as_uint64(s["counts"]).astype(np.float64)
    est = P.estimate_group(Gd, S, s["counts"], l)
    want = E.group_marginal_estimate(g.n, g.src, g.dst, g.w, S, counts / l)
    got = est["marginal"].cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-9)
    assert float(est["group_rwc"][0]) == pytest.approx(E.group_rwc(g.n, g.src, g.dst, g.w, S), rel=1e-9)
    np.testing.assert_allclose(est["hit"].cpu().numpy(), E.hitting_times_to_set(g.n, g.src, g.dst, g.w, S),
                               rtol=1e-9, atol=1e-9)
    so = P.estimate_group(Gd, S, s["counts"], l, stream_ordered=True, max_iter=4000)
    P.workspace_status(so["workspace"])
    assert torch.equal(so["marginal"], est["marginal"]) and torch.equal(so["group_rwc"], est["group_rwc"])


def test_group_estimate_accuracy():
    """ER(300, 6), weighted, S of 4 nodes, 4000 forests: the estimate of H_{S + u} for every u
    is within 1 % mean relative error of its exact value (hitting times to S + u solved
    directly), and the errors match the forests' sampling noise."""
    g = G.erdos_renyi_lcc(300, 6, 41)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 42))
    S = np.array([3, 50, 120, g.n - 1])
    l = 4000
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    s = P.sample_forests(Gd, l, 99, roots=S)
    got = P.estimate_group(Gd, S, s["counts"], l)["marginal"].cpu().numpy()
    exact = np.array([E.group_rwc(g.n, g.src, g.dst, g.w, sorted(set(S.tolist()) | {u})) for u in range(g.n)])
    mre = E.mean_relative_error(exact, got)
    print(f"group marginal MRE at l = {l}: {mre:.4%}")
    assert mre < 0.01


# ------------------------------------------------------------ disconnected graphs -------
def _disconnected():
    """A weighted BA graph, a weighted grid and a path side by side, and two isolated nodes:
    five components; the root set holds one node of each (two in the grid)."""
    ba = G.barabasi_albert(1500, 3, 31)
    ba = ba.with_weights(G.uniform_weights(ba.m, 0.5, 2.0, 32))
    grid = G.grid_with_deletions(900, 0.0, 0)
    grid = grid.with_weights(G.uniform_weights(grid.m, 1.0, 4.0, 33))
    path = G.path_graph(60).with_weights(np.full(59, 1.5, np.float32))
    g = G.disjoint_union([ba, grid, path], isolated=2)
    S = np.array([17, ba.n + 5, ba.n + 800, ba.n + grid.n + 59, g.n - 2, g.n - 1])
    return g, S, (ba.n, grid.n, path.n)


def test_disconnected_build_records_components():
    g, _, (nb, ng, npth) = _disconnected()
    with pytest.raises(P.RWCError) as ei:
        P.Graph(g.n, g.src, g.dst, g.w)
    assert ei.value.status == -6
    Gd = P.Graph(g.n, g.src, g.dst, g.w, allow_disconnected=True)
    assert Gd.components == 5
    comp = Gd.component().cpu().numpy()
    want = np.concatenate([np.zeros(nb), np.full(ng, nb), np.full(npth, nb + ng), [g.n - 2, g.n - 1]])
    np.testing.assert_array_equal(comp, want)
    order = Gd.bfs_order().cpu().numpy()
    assert sorted(order.tolist()) == list(range(g.n))          # every node starts a walk once
    assert order[0] == Gd.csr.pivot_index
    ids = Gd.node_id().cpu().numpy()[order]
    first = np.sum(comp[ids] == comp[Gd.pivot])                 # the pivot's component comes first
    assert (comp[ids[:first]] == comp[Gd.pivot]).all()


@pytest.mark.parametrize("walkers", [1, 8, 64])
def test_disconnected_forests_bit_exact(walkers):
    g, S, _ = _disconnected()
    l = 60
    Gd = P.Graph(g.n, g.src, g.dst, g.w, allow_disconnected=True)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.fastwalk_sample(o, S, 2003, 0, 0, l, want_parents=True, threads=8)
    s = P.sample_forests(Gd, l, 2003, roots=S, walkers_per_tree=walkers, dump=[0, l - 1])
    np.testing.assert_array_equal(P.as_uint64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(P.as_uint64(s["counts_sq"]), ref["visits_sq"])
    np.testing.assert_array_equal(P.as_uint64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(s["parents"].cpu().numpy(), ref["parents"][[0, l - 1]])
    assert int(P.as_uint64(s["total_steps"])[0]) == int(ref["steps"].sum())


def test_disconnected_group_estimate_matches_oracle():
    g, S, _ = _disconnected()
    l = 60
    Gd = P.Graph(g.n, g.src, g.dst, g.w, allow_disconnected=True)
    s = P.sample_forests(Gd, l, 2003, roots=S)
    counts = P.as_uint64(s["counts"]).astype(np.float64)
    est = P.estimate_group(Gd, S, s["counts"], l)
    with np.errstate(invalid="ignore", divide="ignore"):   # the isolated roots' rows of P
        want = E.group_marginal_estimate(g.n, g.src, g.dst, g.w, S, counts / l)
        hs = E.group_rwc(g.n, g.src, g.dst, g.w, S)
        hit = E.hitting_times_to_set(g.n, g.src, g.dst, g.w, S)
    np.testing.assert_allclose(est["marginal"].cpu().numpy(), want, rtol=1e-9)
    assert float(est["group_rwc"][0]) == pytest.approx(hs, rel=1e-9)
    np.testing.assert_allclose(est["hit"].cpu().numpy(), hit, rtol=1e-9, atol=1e-9)


def test_disconnected_graph_is_refused_where_one_root_is_needed():
    """Unrooted sampling, the pivot estimate, trap walks, FastChol, the adjoint and the tuner
    refuse a disconnected CSR on the host; a root set that misses a component is reported by
    the device (the missed component's nodes join the roots, so the launches still end)."""
    g, S, _ = _disconnected()
    Gd = P.Graph(g.n, g.src, g.dst, g.w, allow_disconnected=True)
    calls = [lambda: P.sample_forests(Gd, 4, 1),
             lambda: P.sample_trap_walks(Gd, 2, 1),
             lambda: P.fastchol(Gd),
             lambda: P.autotune(Gd, 64, 1)]
    for call in calls:
        with pytest.raises(P.RWCError) as ei:
            call()
        assert ei.value.status == -6
    counts = P.sample_forests(Gd, 4, 1, roots=S)["counts"]
    with pytest.raises(P.RWCError) as ei:
        P.estimate(Gd, counts, 4)
    assert ei.value.status == -6
    with pytest.raises(P.RWCError) as ei:
        P.backward(Gd, torch.ones(g.n, dtype=torch.float64, device=Gd.device))
    assert ei.value.status == -6
    missing = S[S != g.n - 1]   # the last isolated node holds no root
    for fn in (lambda: P.sample_forests(Gd, 4, 1, roots=missing),
               lambda: P.estimate_group(Gd, missing, counts, 4)):
        with pytest.raises(P.RWCError) as ei:
            fn()
        assert ei.value.status == -6
