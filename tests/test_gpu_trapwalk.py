"""The trap-walk estimator of Lemma 5.1 on the GPU against the oracle's serial trap walks:
visit totals, squared totals and step totals bit for bit under the same keys, on unweighted and
weighted graphs; RWC assembled from them; the step guard reported through the workspace."""
import numpy as np
import pytest

import rwcgen as G
from oracle import exact as E
from oracle import wilson as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _case(name):
    if name == "er1000":
        return G.erdos_renyi_lcc(1000, 8, 1001)
    if name == "ba3000_w":
        g = G.barabasi_albert(3000, 3, 5)
        return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 6))
    if name == "grid_w":
        g = G.grid_with_deletions(400, 0.1, 7)
        return g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, 8))
    if name == "star":
        return G.star_graph(65)
    if name == "k2":
        return G.complete_graph(2)
    raise KeyError(name)


@pytest.mark.parametrize("name,l,begin", [("er1000", 40, 0), ("ba3000_w", 8, 5), ("grid_w", 10, 0), ("star", 30, 0),
                                          ("k2", 50, 3)])
def test_trap_walks_bit_exact(name, l, begin):
    g = _case(name)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.trapwalk_sample(o, o.pivot, 31, 0, begin, l, threads=8)
    r = P.sample_trap_walks(Gd, l, 31, walk_begin=begin)
    np.testing.assert_array_equal(P.as_uint64(r["counts"]), ref["visits"])
    np.testing.assert_array_equal(P.as_uint64(r["counts_sq"]), ref["visits_sq"])
    assert int(P.as_uint64(r["total_steps"])[0]) == ref["steps"]


def test_trap_walks_with_another_trap_and_graph_word():
    g = _case("ba3000_w")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.trapwalk_sample(o, 17, 8, 3, 0, 6, threads=8)
    r = P.sample_trap_walks(Gd, 6, 8, trap=17, graph_index=3)
    np.testing.assert_array_equal(P.as_uint64(r["counts"]), ref["visits"])


def test_trap_walk_rwc_is_the_oracle_assembly():
    """RWC from trap-walk counts through rwc_estimate equals the oracle's Algorithm 1 with the
    same counts (1e-9), and is close to the exact value."""
    g = _case("er1000")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    l = 400
    r = P.sample_trap_walks(Gd, l, 5)
    est = P.estimate(Gd, r["counts"], l)["rwc"].cpu().numpy()
    want = E.fastwalk_estimate(g.n, g.src, g.dst, g.w, Gd.pivot, P.as_uint64(r["counts"]), l)
    np.testing.assert_allclose(est, want, rtol=1e-9)
    exact = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w)
    assert E.mean_relative_error(exact, est) < 0.05


def test_trap_walk_step_guard_is_reported():
    g = _case("grid_w")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    with pytest.raises(P.RWCError) as ei:
        P.sample_trap_walks(Gd, 4, 1, max_steps_per_walk=3)
    assert ei.value.status == -9
