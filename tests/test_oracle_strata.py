"""Pins of the oracle's stratified stack entries (Latin hypercube over the samples), the
variance-reduced estimator at equal trees: every stack entry (u, k) places its word of sample i
in stratum sigma(i) of L = strata, sigma a permutation drawn for that entry.  No GPU.

What pins it: the strata of one entry over the L samples are exactly 0 .. L-1; first
departures then split over the neighbours to within one sample of L p_j (independent draws
miss that by about sqrt(L)); for one sample the strata are uniform and every tree follows the
matrix-tree theorem; the mean visit count stays (calL_v^{-1})_uu (Lemma 5.2) while its
variance across independent seeds drops; the walks still equal cycle popping on the stacks.
"""
import numpy as np
import pytest
import scipy.stats as st

import rwcgen as G
from oracle import exact as E
from oracle import wilson as W

from test_oracle_wilson import _spanning_trees, _tree_of


def _philox_word(k, u, i, g, seed):
    o = W.philox4x32_10([k, u, i, g], [seed & 0xFFFFFFFF, seed >> 32])
    return o[0] | (o[1] << 32)


@pytest.mark.parametrize("L", [2, 3, 5, 7, 64, 100, 1000, 4099])
def test_each_entry_visits_every_stratum_once(L):
    M = (1 << 64) // L
    for (k, u, g, seed) in ((0, 0, 0, 1), (3, 17, 2, 99), (40, 123456, 7, (1 << 40) + 5)):
        words = [W.stack_word(k, u, i, g, seed, L) for i in range(L)]
        assert all(w < L * M for w in words)
        assert sorted(w // M for w in words) == list(range(L))


def test_fewer_than_two_strata_is_the_plain_draw():
    for i in range(20):
        plain = _philox_word(2, 11, i, 3, 77)
        assert W.stack_word(2, 11, i, 3, 77, 0) == plain
        assert W.stack_word(2, 11, i, 3, 77, 1) == plain
        assert W.stack_word(2, 11, i, 3, 77, 64) != plain


def test_stratified_first_departures_split_evenly():
    # star centre of degree 8, L = 1024 a multiple of 8 and a power of two: exactly L/8 each
    g = G.star_graph(9)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    for k in range(4):
        picks = [W.random_neighbor(csr, 0, k, i, 0, 5, strata=1024) for i in range(1024)]
        np.testing.assert_array_equal(np.bincount(np.asarray(picks) - 1, minlength=8), np.full(8, 128))


def test_stratified_weighted_departures_track_the_weights():
    w = np.array([0.5, 1.0, 2.0, 4.0, 0.75, 1.25], dtype=np.float32)
    g = G.star_graph(7).with_weights(w)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    L = 1000
    p = w.astype(np.float64) / w.sum()
    worst_iid = 0.0
    for k in range(6):
        strat = np.bincount(np.asarray([W.random_neighbor(csr, 0, k, i, 0, 8, strata=L) for i in range(L)]) - 1,
                            minlength=6)
        iid = np.bincount(np.asarray([W.random_neighbor(csr, 0, k, i, 0, 8) for i in range(L)]) - 1, minlength=6)
        assert np.max(np.abs(strat - L * p)) <= 2.0
        worst_iid = max(worst_iid, float(np.max(np.abs(iid - L * p))))
    assert worst_iid > 2.0      # independent draws do not balance like this


def test_one_sample_sees_uniform_strata():
    L, i = 6, 2
    M = (1 << 64) // L
    words = [W.stack_word(k, u, i, 0, 31, L) for u in range(300) for k in range(40)]
    strata = np.asarray([w // M for w in words])
    assert st.chisquare(np.bincount(strata, minlength=L)).pvalue > 1e-3
    frac = np.asarray([(w - (w // M) * M) / M for w in words])
    assert st.kstest(frac, "uniform").pvalue > 1e-3


def test_stratified_trees_follow_matrix_tree_theorem():
    """For one sample index the tree is a weighted uniform spanning tree; seeds are independent."""
    src = np.array([0, 0, 1, 1, 2, 3, 4, 2], dtype=np.int32)
    dst = np.array([1, 2, 2, 3, 4, 4, 5, 5], dtype=np.int32)
    g = G.EdgeList(6, src, dst, np.array([0.5, 2.0, 1.0, 4.0, 1.5, 0.75, 3.0, 1.0], np.float32))
    edges = [(int(min(a, b)), int(max(a, b))) for a, b in zip(g.src, g.dst)]
    edge_index = {e: i for i, e in enumerate(edges)}
    trees = _spanning_trees(g.n, edges)
    weight = np.array([np.prod(g.w.astype(np.float64)[list(t)]) for t in trees])
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    root = csr.pivot
    idx = {t: i for i, t in enumerate(trees)}
    nseeds = 30 * len(trees) + 2000
    counts = np.zeros(len(trees))
    L = 16
    for s in range(nseeds):
        r = W.fastwalk_sample(csr, root, 1000 + s, 0, s % L, 1, want_parents=True, strata=L)
        counts[idx[_tree_of(r["parents"][0], root, edge_index)]] += 1
    assert st.chisquare(counts, weight / weight.sum() * nseeds).pvalue > 1e-3


def _per_seed_means(csr, v, L, seeds, strata):
    out = np.empty((len(seeds), csr.n))
    for r, s in enumerate(seeds):
        res = W.fastwalk_sample(csr, v, s, 0, 0, L, strata=strata)
        out[r] = res["visits"].astype(float) / L
    return out


@pytest.mark.parametrize("case", ["er30_w", "grid36"])
def test_stratified_counts_unbiased_with_lower_variance(case):
    """Lemma 5.2 holds for the stratified mean (z-test over independent seeds), and its
    variance across seeds is well below that of independent draws at the same l."""
    if case == "er30_w":
        g = G.erdos_renyi_lcc(30, 4, 9)
        g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 10))
    else:
        g = G.grid_with_deletions(36, 0.0, 0)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    v = csr.pivot
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    L, R = 64, 400
    strat = _per_seed_means(csr, v, L, range(5000, 5000 + R), L)
    iid = _per_seed_means(csr, v, L, range(5000, 5000 + R), 0)
    mask = np.arange(g.n) != v
    mean = strat.mean(0)[mask]
    sd = strat.std(0, ddof=1)[mask]
    moving = sd > 0
    z = (mean[moving] - t[mask][moving]) / (sd[moving] / np.sqrt(R))
    assert np.max(np.abs(z)) < 5.0
    ratio = strat.var(0, ddof=1)[mask].sum() / iid.var(0, ddof=1)[mask].sum()
    assert ratio < 0.85, ratio


def test_stratified_runs_split_and_reject_out_of_range_samples():
    g = G.erdos_renyi_lcc(40, 5, 3)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    whole = W.fastwalk_sample(csr, csr.pivot, 9, 0, 0, 32, strata=32)
    a = W.fastwalk_sample(csr, csr.pivot, 9, 0, 0, 16, strata=32)
    b = W.fastwalk_sample(csr, csr.pivot, 9, 0, 16, 16, strata=32)
    thr = W.fastwalk_sample(csr, csr.pivot, 9, 0, 0, 32, strata=32, threads=4)
    for key in ("visits", "visits_sq"):
        np.testing.assert_array_equal(whole[key], a[key] + b[key])
        np.testing.assert_array_equal(whole[key], thr[key])
    np.testing.assert_array_equal(whole["hash"], np.concatenate([a["hash"], b["hash"]]))
    plain = W.fastwalk_sample(csr, csr.pivot, 9, 0, 0, 32)
    assert not np.array_equal(whole["hash"], plain["hash"])
    with pytest.raises(RuntimeError):
        W.fastwalk_sample(csr, csr.pivot, 9, 0, 20, 16, strata=32)
    with pytest.raises(RuntimeError):
        W.fastwalk_sample(csr, csr.pivot, 9, 0, 0, 4, strata=(1 << 31) + 1)
