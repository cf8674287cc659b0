"""Full-size checks in the launch configurations bench.py times.

BA(n = 1e6, m = 5), 10^4 trees: the automatic plan (64-walker teams, one batch) must
reproduce the oracle's trees: parent arrays of sampled trees, the checksum of every tree and
the visit totals, plus properties that hold at any size.  The 256-graph batch in its
persistent, hipGraph-captured launch: every tree and every visit total of every graph against
the oracle and against plain per-graph launches.  R-MAT scale 23 (largest component, weighted),
5000 trees in a persistent launch: every tree and the visit totals against the oracle, and the
adjoint for 1000 targets against the oracle's stored sparse evaluation.
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


def test_ba1m_bench_configuration_matches_oracle_on_every_tree():
    """All 10^4 trees of the bench's launch against the oracle run over the host cores: every
    tree checksum, the visit totals and their squares, bit for bit (the oracle needs about
    90 s on 16 threads)."""
    import os
    g = G.barabasi_albert(1_000_000, 5, 1002)
    l, seed = 10_000, 2002
    Gd = P.Graph(g.n, g.src, g.dst)
    dump = [0, 9_999]
    s = P.sample_forests(Gd, l, seed, dump=dump)
    assert s["walkers_per_tree"] == 64 and s["trees_in_flight"] == l     # the bench's team plan
    _check_sampled_trees(g, s, l, seed, [0, 1, 2047, 2048, 5001, 9_999], dump)
    o = W.OracleCSR(g.n, g.src, g.dst, g.w)
    ref = W.fastwalk_sample(o, o.pivot, seed, 0, 0, l, threads=max(1, min(16, os.cpu_count() or 1)))
    np.testing.assert_array_equal(P.as_uint64(s["tree_hash"][0]), ref["hash"])
    np.testing.assert_array_equal(P.as_uint64(s["counts"]), ref["visits"])
    np.testing.assert_array_equal(P.as_uint64(s["counts_sq"]), ref["visits_sq"])
    assert int(P.as_uint64(s["total_steps"])[0]) == int(ref["steps"].sum())


# ---------------------------------------------------------------------------------------
# The 256-graph batch in the bench's launch (persistent, hipGraph-captured, automatic plan):
# every tree checksum and every visit total of every graph against the oracle, and against
# one plain launch per graph.  The oracle's 2.8e10 steps are split into chunks of about equal
# work (from the GPU's step totals), one test per chunk, so no test runs long.
# ---------------------------------------------------------------------------------------
BATCH_CHUNKS = 6


@pytest.fixture(scope="module")
def batch256():
    gl = G.batch_mix(256, 1e3, 1e5, seed=1003)
    l, seed = 1000, 2003
    dev = [P.Graph(g.n, g.src, g.dst, g.w) for g in gl]
    s = P.sample_forests(dev, l, seed, persistent=True, capture=True, want_sq=True)
    out = {"gl": gl, "dev": dev, "l": l, "seed": seed, "hash": P.as_uint64(s["tree_hash"]).copy(),
           "counts": P.as_uint64(s["counts"]).copy(), "counts_sq": P.as_uint64(s["counts_sq"]).copy(),
           "steps": P.as_uint64(s["total_steps"]).copy(), "off": np.concatenate([[0], np.cumsum([g.n for g in gl])])}
    # contiguous chunks of graphs with about equal oracle work
    cum = np.cumsum(out["steps"].astype(np.float64))
    bounds = np.searchsorted(cum, cum[-1] * np.arange(1, BATCH_CHUNKS) / BATCH_CHUNKS)
    out["chunks"] = np.split(np.arange(len(gl)), bounds)
    del s
    P.release_cached_graphs()
    return out


def test_batch256_invariants_and_plain_launches_bit_identical(batch256):
    """Per-tree invariants of every graph, and the batched launch's outputs equal to 256 plain
    per-graph launches (the acceptance of the batched form: the same outputs either way), bit
    for bit."""
    b = batch256
    for gi, g in enumerate(b["gl"]):
        c = b["counts"][b["off"][gi]:b["off"][gi + 1]]
        piv = int(b["dev"][gi].pivot)
        assert c[piv] == 0 and (np.delete(c, piv) >= b["l"]).all(), f"graph {gi}"
        assert int(c.sum()) == int(b["steps"][gi])
    ws = None
    for gi, Gd in enumerate(b["dev"]):
        r = P.sample_forests(Gd, b["l"], b["seed"], graph_index_base=gi, want_sq=True, workspace=ws)
        ws = r["workspace"]
        np.testing.assert_array_equal(P.as_uint64(r["tree_hash"][0]), b["hash"][gi], err_msg=f"graph {gi}")
        np.testing.assert_array_equal(P.as_uint64(r["counts"]), b["counts"][b["off"][gi]:b["off"][gi + 1]])
        np.testing.assert_array_equal(P.as_uint64(r["counts_sq"]), b["counts_sq"][b["off"][gi]:b["off"][gi + 1]])


@pytest.mark.parametrize("chunk", range(BATCH_CHUNKS))
def test_batch256_every_tree_matches_oracle(batch256, chunk):
    import os
    b = batch256
    threads = max(1, min(16, os.cpu_count() or 1))
    for gi in b["chunks"][chunk]:
        g = b["gl"][gi]
        o = W.OracleCSR(g.n, g.src, g.dst, g.w)
        ref = W.fastwalk_sample(o, o.pivot, b["seed"], int(gi), 0, b["l"], threads=threads)
        np.testing.assert_array_equal(b["hash"][gi], ref["hash"], err_msg=f"graph {gi}")
        np.testing.assert_array_equal(b["counts"][b["off"][gi]:b["off"][gi + 1]], ref["visits"])
        np.testing.assert_array_equal(b["counts_sq"][b["off"][gi]:b["off"][gi + 1]], ref["visits_sq"])
        assert int(b["steps"][gi]) == int(ref["steps"].sum())


# ---------------------------------------------------------------------------------------
# R-MAT scale 23 (largest component, w ~ U[1, 4]), 5000 trees in the bench's persistent
# launch: every tree checksum, the visit totals and their squares against the oracle (in
# three sample-range chunks whose integer sums add up), and the adjoint for 1000 targets
# (k = 64) against the oracle's sparse evaluation stored in tests/golden.
# ---------------------------------------------------------------------------------------
RMAT_CHUNKS = 3
# Adjoint tolerances.  Both sides stop each solve at relative residual 1e-11 (the GPU with FP32
# search directions but FP64 residuals, so its stopping test is as strict as the oracle's).
# The gradient here is dominated by its common term 2 trGL^ (about 437.8 at every edge); the
# edge-specific part varies by about 1.6 over the stored edges.  The solution error is at most
# cond(L_v) * 1e-11 relative; measured, the two sides agree to 7e-15 of max |grad| and to 2e-12
# of the edge-specific spread, so the bounds below keep three orders of magnitude of margin on
# both: the full value to 1e-11 of max |grad|, the edge-specific part to 1e-9 of its spread.
RMAT_ADJOINT_TOL = 1e-11
RMAT_ADJOINT_CENTRED_TOL = 1e-9


@pytest.fixture(scope="module")
def rmat23():
    g = G.rmat_lcc(23, 5, 0.57, 0.19, 0.19, 1005)
    g = g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, 1006))
    l, seed = 5000, 2005
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    dump = [3, 4999]
    s = P.sample_forests(Gd, l, seed, dump=dump, persistent=True, want_sq=True)
    print(f"R-MAT LCC n={g.n} m={g.m}: {s['walkers_per_tree']} walkers x {s['trees_in_flight']} trees, "
          f"{s['batches']} batches, {s['walk_kernel']}, {s['starts']} starts")
    out = {"g": g, "Gd": Gd, "l": l, "seed": seed, "dump": dump, "parents": s["parents"].cpu().numpy(),
           "hash": P.as_uint64(s["tree_hash"][0]).copy(), "counts": P.as_uint64(s["counts"]).copy(),
           "counts_sq": P.as_uint64(s["counts_sq"]).copy(), "steps": int(P.as_uint64(s["total_steps"])[0]),
           "o": W.OracleCSR(g.n, g.src, g.dst, g.w), "acc": {}}
    del s
    return out


def test_rmat23_launch_and_dumped_trees(rmat23):
    r = rmat23
    o = r["o"]
    assert r["counts"][o.pivot] == 0
    mask = np.ones(r["g"].n, dtype=bool)
    mask[o.pivot] = False
    assert (r["counts"][mask] >= r["l"]).all()
    assert int(r["counts"].sum()) == r["steps"]
    for j, i in enumerate(r["dump"]):
        ref = W.fastwalk_sample(o, o.pivot, r["seed"], 0, i, 1, want_parents=True)
        np.testing.assert_array_equal(r["parents"][j], ref["parents"][0])
        assert int(r["hash"][i]) == int(ref["hash"][0])


@pytest.mark.parametrize("chunk", range(RMAT_CHUNKS))
def test_rmat23_every_tree_matches_oracle(rmat23, chunk):
    """Samples of this chunk: every checksum; the oracle's visit totals of all chunks add up to
    the GPU's totals and squared totals (checked once the last chunk has run)."""
    import os
    r = rmat23
    o = r["o"]
    lo, hi = chunk * r["l"] // RMAT_CHUNKS, (chunk + 1) * r["l"] // RMAT_CHUNKS
    ref = W.fastwalk_sample(o, o.pivot, r["seed"], 0, lo, hi - lo, threads=max(1, min(16, os.cpu_count() or 1)))
    np.testing.assert_array_equal(r["hash"][lo:hi], ref["hash"])
    r["acc"][chunk] = (ref["visits"], ref["visits_sq"], int(ref["steps"].sum()))
    if len(r["acc"]) == RMAT_CHUNKS:
        v = sum(a[0] for a in r["acc"].values())
        v2 = sum(a[1] for a in r["acc"].values())
        np.testing.assert_array_equal(r["counts"], v)
        np.testing.assert_array_equal(r["counts_sq"], v2)
        assert r["steps"] == sum(a[2] for a in r["acc"].values())


def _rmat23_adjoint_fixture():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "rmat23_adjoint_grad.txt")
    rows = [line.split("|") for line in open(path) if not line.startswith("#")]
    return (np.array([int(a) for a, _, _, _ in rows]), np.array([int(b) for _, b, _, _ in rows]),
            np.array([int(c) for _, _, c, _ in rows]), np.array([float(d) for _, _, _, d in rows]))


def test_rmat23_adjoint_matches_oracle_fixture(rmat23):
    """The adjoint for 1000 targets (g = 1, k = 64 probes, probe seed 2006) at the 24 edges the
    oracle evaluated (tests/golden/make_rmat23_adjoint.py: sparse CG solves to 1e-11), in full
    and with the common term taken out."""
    r = rmat23
    g = r["g"]
    edges, a, b, want = _rmat23_adjoint_fixture()
    np.testing.assert_array_equal(g.src[edges], a)
    np.testing.assert_array_equal(g.dst[edges], b)
    t = np.random.default_rng(7).choice(g.n, size=1000, replace=False).astype(np.int32)
    res = P.backward(r["Gd"], P.dense_g(g.n, t, np.ones(1000), "cuda"), k=64, seed=2006, tol=1e-11)
    grad = res["grad_w"].cpu().numpy()
    scale = np.abs(want).max()
    err = np.abs(grad[edges] - want)
    # the edge-specific part, with the common term 2 trGL^ (about 437.8 here) taken out
    cen = np.abs((grad[edges] - grad[edges].mean()) - (want - want.mean()))
    print(f"R-MAT adjoint: {res['iters']} iterations, max |err| = {err.max():.3e} "
          f"({err.max() / scale:.3e} of max |grad|), centred max |err| = {cen.max():.3e} "
          f"(spread {np.ptp(want):.3e})")
    assert err.max() <= RMAT_ADJOINT_TOL * scale
    assert cen.max() <= RMAT_ADJOINT_CENTRED_TOL * np.ptp(want)
    assert np.isfinite(grad).all()
    assert abs(np.dot(g.w, grad)) <= 1e-6 * np.abs(g.w * grad).sum()


def test_ba20k_rwc_within_error_of_exact_at_1e4_trees():
    """BA(20 000, 5) (the exact-checkable copy of the bench graph), 10^4 trees: RWC against the
    exact FP64 values stored by tests/golden/make_ba20k_exact.py.  The pivot's value comes from
    the solve alone (relative 1e-9); elsewhere the mean relative error at this sample count is
    below 1 % (about 0.3 % expected from the per-node standard errors) and the errors are
    consistent with the estimated standard errors."""
    import os
    from oracle import exact as E
    path = os.path.join(os.path.dirname(__file__), "golden", "ba20k_exact_rwc.txt")
    rows = [line.split("|") for line in open(path) if not line.startswith("#")]
    nodes = np.array([int(a) for a, _ in rows])
    exact = np.array([float(b) for _, b in rows])
    g = G.barabasi_albert(20_000, 5, 1002)
    Gd = P.Graph(g.n, g.src, g.dst)
    s = P.sample_forests(Gd, 10_000, 2002)
    est = P.estimate(Gd, s["counts"], 10_000, counts_sq=s["counts_sq"], want_stderr=True)
    got = est["rwc"].cpu().numpy()[nodes]
    se = est["stderr"].cpu().numpy()[nodes]
    v = Gd.pivot
    iv = int(np.flatnonzero(nodes == v)[0])
    assert abs(got[iv] - exact[iv]) <= 1e-9 * exact[iv]
    mask = nodes != v
    mre = E.mean_relative_error(exact[mask], got[mask])
    print(f"BA(20000, 5), l = 10^4: MRE {mre:.4%} over {mask.sum()} sampled nodes")
    assert mre < 0.01
    z = np.abs(got[mask] - exact[mask]) / se[mask]
    assert np.mean(z > 4) < 0.005
