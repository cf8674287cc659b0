"""Full-size checks in the launch configuration bench.py times.

BA(n = 1e6, m = 5), 10^4 trees: the automatic plan (walker teams, several batches) must
reproduce the oracle's trees one by one for sampled sample indices (checksum and parent
array), plus properties that hold at any size.  R-MAT scale 23 (largest component, weighted):
the same, with fewer trees, and the adjoint's Euler identity.
"""
import numpy as np
import pytest

import rwcgen as G
from oracle import wilson as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _check_sampled_trees(g, s, l, seed, picks, dump):
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    hashes = P.as_uint64(s["tree_hash"][0])
    for i in picks:
        ref = W.fastwalk_sample(o, o.pivot, seed, 0, i, 1, want_parents=True)
        assert int(hashes[i]) == int(ref["hash"][0]), f"tree {i}"
        if i in dump:
            np.testing.assert_array_equal(s["parents"][dump.index(i)].cpu().numpy(), ref["parents"][0])
    counts = P.as_uint64(s["counts"])
    piv = o.pivot
    assert counts[piv] == 0
    mask = np.ones(g.n, dtype=bool)
    mask[piv] = False
    assert (counts[mask] >= l).all()          # every non-root node departs at least once per tree
    assert int(counts.sum()) == int(P.as_uint64(s["total_steps"])[0])


def test_ba1m_bench_configuration_sampled_trees():
    g = G.barabasi_albert(1_000_000, 5, 1002)
    l, seed = 10_000, 2002
    Gd = P.Graph(g.n, g.src, g.dst)
    dump = [0, 9_999]
    s = P.sample_forests(Gd, l, seed, dump=dump)
    assert s["walkers_per_tree"] == 64 and s["trees_in_flight"] == l     # the bench's team plan
    _check_sampled_trees(g, s, l, seed, [0, 1, 2047, 2048, 5001, 9_999], dump)


def test_rmat_scale23_sampled_trees_and_adjoint():
    g = G.rmat_lcc(23, 5, 0.57, 0.19, 0.19, 1005)
    g = g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, 1006))
    l, seed = 256, 2005
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    dump = [3]
    s = P.sample_forests(Gd, l, seed, dump=dump, persistent=True)
    _check_sampled_trees(g, s, l, seed, [0, 3, 255], dump)
    rng = np.random.default_rng(7)
    t = rng.choice(g.n, size=1000, replace=False).astype(np.int32)
    res = P.backward(Gd, t, np.ones(1000), k=64, seed=2006, tol=1e-8)
    grad = res["grad_w"].cpu().numpy()
    assert np.isfinite(grad).all()
    assert abs(np.dot(g.w, grad)) <= 1e-6 * np.abs(g.w * grad).sum()
