"""Pins of the serial FastWalk oracle (Algorithm 3) against the mathematics (no GPU)."""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats as st

import rwcgen as G
from oracle import exact as E
from oracle import wilson as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox4x32-10 ------
def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c, k, o = line.split("|")
            rows.append(([int(x, 16) for x in c.split()], [int(x, 16) for x in k.split()],
                         tuple(int(x, 16) for x in o.split())))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert W.philox4x32_10(ctr, key) == out


def test_philox_matches_rocrand_engine(tmp_path):
    """2000 random counters/keys against rocRAND's independent Philox4x32-10 engine."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "ref"
    subprocess.run([hipcc, "-O1", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", str(exe)], check=True,
                   capture_output=True)
    rng = np.random.default_rng(7)
    words = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)
    words[:50, 0] = np.arange(50)           # small departure counts, as the sampler uses
    words[50:100, 2:4] = 0
    inp = "\n".join(" ".join(str(int(x)) for x in r) for r in words) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    ref = [tuple(int(x) for x in line.split()) for line in res.stdout.strip().splitlines()]
    got = [W.philox4x32_10(r[:4], r[4:]) for r in words]
    assert got == ref


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 0 and 1 (state increments by the golden gamma
    # before mixing): these are the published first values of the generator.
    assert W.splitmix64(0) == 0xE220A8397B1DCDAF
    assert W.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


# ------------------------------------------------------------------ selection law ------
def test_weighted_selection_is_proportional_to_weight():
    w = np.array([0.5, 1.0, 2.0, 4.0, 0.75, 1.25], dtype=np.float32)
    g = G.star_graph(7).with_weights(w)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    draws = [W.random_neighbor(csr, 0, k, s, 0, 99) for s in range(60) for k in range(500)]
    counts = np.bincount(np.asarray(draws) - 1, minlength=6)
    p = st.chisquare(counts, w / w.sum() * counts.sum()).pvalue
    assert p > 1e-3


def test_unit_weights_reduce_to_unweighted_rule():
    g = G.erdos_renyi_lcc(200, 6, 3)
    a = W.OracleCSR(g.n, g.src, g.dst, None)
    b = W.OracleCSR(g.n, g.src, g.dst, np.ones(g.m, dtype=np.float32))
    ra = W.fastwalk_sample(a, a.pivot, 5, 0, 0, 40)
    rb = W.fastwalk_sample(b, b.pivot, 5, 0, 0, 40)
    for key in ("visits", "visits_sq", "steps", "hash"):
        np.testing.assert_array_equal(ra[key], rb[key])


# ------------------------------------------------------------ tree distribution -------
def _spanning_trees(n, edges):
    """All spanning trees by brute force over (n-1)-subsets of the edges."""
    out = []
    for sub in itertools.combinations(range(len(edges)), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        ok = True
        for e in sub:
            a, b = edges[e]
            ra, rb = find(a), find(b)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
        if ok:
            out.append(frozenset(sub))
    return out


def _tree_of(parents, root, edge_index):
    return frozenset(edge_index[(min(u, p), max(u, p))] for u, p in enumerate(parents) if u != root)


@pytest.mark.parametrize("case", ["K4", "K5", "grid3x3", "weighted6"])
def test_tree_distribution_matches_matrix_tree_theorem(case):
    if case == "K4":
        g = G.complete_graph(4)
    elif case == "K5":
        g = G.complete_graph(5)
    elif case == "grid3x3":
        g = G.grid_with_deletions(9, 0.0, 0)
    else:
        src = np.array([0, 0, 1, 1, 2, 3, 4, 2], dtype=np.int32)
        dst = np.array([1, 2, 2, 3, 4, 4, 5, 5], dtype=np.int32)
        g = G.EdgeList(6, src, dst, np.array([0.5, 2.0, 1.0, 4.0, 1.5, 0.75, 3.0, 1.0], np.float32))
    edges = [(int(min(a, b)), int(max(a, b))) for a, b in zip(g.src, g.dst)]
    edge_index = {e: i for i, e in enumerate(edges)}
    w = np.ones(g.m) if g.w is None else g.w.astype(np.float64)
    trees = _spanning_trees(g.n, edges)
    weight = np.array([np.prod(w[list(t)]) for t in trees])
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    root = csr.pivot
    L = E.laplacian(E.adjacency(g.n, g.src, g.dst, g.w))
    keep = [i for i in range(g.n) if i != root]
    assert weight.sum() == pytest.approx(np.linalg.det(L[np.ix_(keep, keep)]), rel=1e-9)
    nsamp = 30 * len(trees) + 2000
    r = W.fastwalk_sample(csr, root, 1234, 0, 0, nsamp, want_parents=True)
    idx = {t: i for i, t in enumerate(trees)}
    counts = np.zeros(len(trees))
    for par in r["parents"]:
        counts[idx[_tree_of(par, root, edge_index)]] += 1
    p = st.chisquare(counts, weight / weight.sum() * nsamp).pvalue
    assert p > 1e-3


def test_edge_marginals_follow_kirchhoff():
    """P(e in T) = w_e R_e for a weighted uniform-by-weight spanning tree."""
    g = G.erdos_renyi_lcc(12, 4, 2)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 3))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    nsamp = 20000
    r = W.fastwalk_sample(csr, csr.pivot, 77, 0, 0, nsamp, want_parents=True)
    Lp = E.laplacian_pinv(E.laplacian(E.adjacency(g.n, g.src, g.dst, g.w)))
    for e in range(g.m):
        a, b = int(g.src[e]), int(g.dst[e])
        inside = np.mean((r["parents"][:, a] == b) | (r["parents"][:, b] == a))
        pe = g.w[e] * (Lp[a, a] + Lp[b, b] - 2 * Lp[a, b])
        var = max(pe * (1 - pe), 0.0)           # bridges have pe = 1 up to rounding
        assert abs(inside - pe) < 5 * np.sqrt(var / nsamp) + 1e-9


# ------------------------------------------------------------ visits and steps --------
def test_expected_visits_lemma_5_2():
    """E[visits to u in one Wilson tree rooted at v] = (calL_v^{-1})_uu (Lemma 5.2)."""
    g = G.erdos_renyi_lcc(30, 4, 9)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 10))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    v = csr.pivot
    l = 40000
    r = W.fastwalk_sample(csr, v, 2024, 0, 0, l, threads=4)
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    mean = r["visits"].astype(float) / l
    var = r["visits_sq"].astype(float) / l - mean ** 2
    mask = np.arange(g.n) != v
    z = (mean[mask] - t[mask]) / np.sqrt(var[mask] / l)
    assert np.max(np.abs(z)) < 5.0
    assert r["visits"][v] == 0


@pytest.mark.parametrize("kind,n", [("K", 7), ("C", 9), ("ER", 25)])
def test_expected_steps_theorem_5_7(kind, n):
    g = {"K": lambda: G.complete_graph(n), "C": lambda: G.cycle_graph(n),
         "ER": lambda: G.erdos_renyi_lcc(n, 4, 5)}[kind]()
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    v = csr.pivot
    l = 20000
    r = W.fastwalk_sample(csr, v, 31, 0, 0, l, threads=4)
    s = r["steps"].astype(float)
    exp = E.expected_steps_per_tree(g.n, g.src, g.dst, None, v)
    assert abs(s.mean() - exp) < 5 * s.std() / np.sqrt(l)
    assert s.sum() == r["visits"].sum()


def test_star_rooted_at_centre_is_deterministic():
    g = G.star_graph(9)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    assert csr.pivot == 0
    r = W.fastwalk_sample(csr, 0, 1, 0, 0, 5, want_parents=True)
    assert (r["steps"] == 8).all()
    np.testing.assert_array_equal(r["visits"], np.array([0] + [5] * 8, dtype=np.uint64))
    assert (r["parents"][:, 1:] == 0).all() and (r["parents"][:, 0] == -1).all()


def test_order_and_split_independence():
    """Stack-keyed choices make the forest independent of the start order (cycle popping),
    of thread splits and of sample-range chunking."""
    g = G.barabasi_albert(300, 2, 4)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 5))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    v = csr.pivot
    base = W.fastwalk_sample(csr, v, 8, 3, 0, 30, want_parents=True)
    for s in range(3):
        perm = np.random.default_rng(s).permutation(g.n)
        r = W.fastwalk_sample(csr, v, 8, 3, 0, 30, order=perm, want_parents=True)
        for key in ("visits", "visits_sq", "steps", "hash", "parents"):
            np.testing.assert_array_equal(r[key], base[key])
    rt = W.fastwalk_sample(csr, v, 8, 3, 0, 30, threads=3)
    np.testing.assert_array_equal(rt["visits"], base["visits"])
    a = W.fastwalk_sample(csr, v, 8, 3, 0, 11)
    b = W.fastwalk_sample(csr, v, 8, 3, 11, 19)
    np.testing.assert_array_equal(a["visits"] + b["visits"], base["visits"])
    np.testing.assert_array_equal(np.concatenate([a["hash"], b["hash"]]), base["hash"])
    # a different graph word gives a different forest
    other = W.fastwalk_sample(csr, v, 8, 4, 0, 30)
    assert not np.array_equal(other["hash"], base["hash"])


def test_tree_hash_definition():
    g = G.erdos_renyi_lcc(50, 4, 8)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    r = W.fastwalk_sample(csr, csr.pivot, 3, 0, 0, 4, want_parents=True)
    for s in range(4):
        h = 0
        for u, p in enumerate(r["parents"][s]):
            if u != csr.pivot:
                h = (h + W.splitmix64((u << 32) | int(p))) % (1 << 64)
        assert h == int(r["hash"][s])


def test_estimate_accuracy_er1000():
    """ER(1000, 8) with 2000 trees: the FastWalk estimate is within a few percent MRE of the
    exact RWC (the accuracy the GPU path inherits bit-for-bit)."""
    g = G.erdos_renyi_lcc(1000, 8, 1001)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    l = 2000
    r = W.fastwalk_sample(csr, csr.pivot, 2001, 0, 0, l, threads=8)
    est = E.fastwalk_estimate(g.n, g.src, g.dst, None, csr.pivot, r["visits"], l)
    exact = E.rwc_laplacian_pinv(g.n, g.src, g.dst, None)
    assert E.mean_relative_error(exact, est) < 0.03


# ------------------------------------------------------------ cycle popping -----------
def _cycle_popping(csr, roots, seed, graph, sample, strata=0):
    """Wilson's cycle-popping construction, written independently of the walk: node u's k-th
    arrow is the neighbour RandomNeighbor chooses at its k-th departure; while the current top
    arrows of the non-root nodes contain a cycle, pop it (every node on it moves to its next
    arrow); the arrows left form the forest.  A non-root's departures are its pops plus one."""
    n = csr.n
    is_root = np.zeros(n, dtype=bool)
    is_root[list(roots)] = True
    top = np.zeros(n, dtype=np.int64)
    cur = np.full(n, -1, dtype=np.int64)
    for u in range(n):
        if not is_root[u]:
            cur[u] = W.random_neighbor(csr, u, 0, sample, graph, seed, strata)
    while True:
        state = np.zeros(n, dtype=np.int8)      # 0 unseen, 1 on the current chain, 2 done
        cycles = []
        for s0 in range(n):
            if is_root[s0] or state[s0]:
                continue
            chain = []
            u = s0
            while not is_root[u] and state[u] == 0:
                state[u] = 1
                chain.append(u)
                u = cur[u]
            if not is_root[u] and state[u] == 1:       # closed a new cycle at u
                cycles.append(chain[chain.index(u):])
            for x in chain:
                state[x] = 2
        if not cycles:
            break
        for cyc in cycles:                              # disjoint: pop them all
            for u in cyc:
                top[u] += 1
                cur[u] = W.random_neighbor(csr, u, int(top[u]), sample, graph, seed, strata)
    dep = np.where(is_root, 0, top + 1).astype(np.uint64)
    par = np.where(is_root, -1, cur).astype(np.int32)
    return dep, par


@pytest.mark.parametrize("roots,strata", [(None, 0), ((0, 7), 0), ((3, 11, 19, 25), 0), (None, 24), ((0, 7), 24)])
def test_walks_equal_cycle_popping(roots, strata):
    """The oracle's loop-erased walks pop exactly the cycles of the stack picture: same forest,
    same departure count at every node, for one root and for root sets, with independent or
    stratified stack entries."""
    g = G.erdos_renyi_lcc(30, 4, 12)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 13))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    S = [csr.pivot] if roots is None else list(roots)
    r = W.fastwalk_sample(csr, S if roots else csr.pivot, 404, 2, 10, 12, want_parents=True, strata=strata)
    tot = np.zeros(g.n, dtype=np.uint64)
    for s in range(12):
        dep, par = _cycle_popping(csr, S, 404, 2, 10 + s, strata)
        np.testing.assert_array_equal(r["parents"][s], par)
        assert int(r["steps"][s]) == int(dep.sum())
        tot += dep
    np.testing.assert_array_equal(r["visits"], tot)


def test_algorithm3_visit_bookkeeping_equals_departures():
    """Algorithm 3's count (+1 at a walk start, +1 per arrival, -1 at the arrival in the tree),
    replayed on the oracle's own forests, is the departure count it reports."""
    g = G.barabasi_albert(40, 2, 3)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    v = csr.pivot
    r = W.fastwalk_sample(csr, v, 9, 0, 0, 8)
    total = np.zeros(g.n, dtype=np.int64)
    for s in range(8):
        in_tree = np.zeros(g.n, dtype=bool)
        in_tree[v] = True
        nxt = np.full(g.n, -1)
        dep = np.zeros(g.n, dtype=np.int64)
        vis = np.zeros(g.n, dtype=np.int64)
        for j in range(g.n):
            if in_tree[j]:
                continue
            u = j
            vis[u] += 1
            while not in_tree[u]:
                nxt[u] = W.random_neighbor(csr, u, int(dep[u]), s, 0, 9)
                dep[u] += 1
                u = nxt[u]
                vis[u] += 1
            vis[u] -= 1
            u = j
            while not in_tree[u]:
                in_tree[u] = True
                u = nxt[u]
        total += vis
    np.testing.assert_array_equal(r["visits"].astype(np.int64), total)


# ------------------------------------------------------------ root sets (forests) -----
def _rooted_forests(n, edges, S):
    """Spanning forests in which every tree holds exactly one node of S: the spanning trees of
    the graph with S merged into one node, by brute force over (n - |S|)-subsets of edges."""
    out = []
    for sub in itertools.combinations(range(len(edges)), n - len(S)):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        for s in S[1:]:
            parent[find(s)] = find(S[0])
        ok = True
        for e in sub:
            a, b = edges[e]
            ra, rb = find(a), find(b)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
        if ok:
            out.append(frozenset(sub))
    return out


@pytest.mark.parametrize("case", ["grid3x3", "weighted6", "K5", "disconnected"])
def test_forest_distribution_matches_matrix_forest_theorem(case):
    """Forests rooted at S: the sum over them of prod w_e is det(L_S) (the matrix-tree theorem
    with S merged, or the all-minors form), and the sampled forests follow prod w_e (chi^2).
    The disconnected case (K4, a weighted 4-cycle and an isolated node, one root in each
    component and a second one in the cycle) has one factor of det(L_S) per component."""
    if case == "grid3x3":
        g, S = G.grid_with_deletions(9, 0.0, 0), [0, 8]
    elif case == "K5":
        g, S = G.complete_graph(5), [1, 3]
    elif case == "disconnected":
        c4 = G.cycle_graph(4).with_weights(np.array([0.5, 2.0, 1.0, 3.0], np.float32))
        k4 = G.complete_graph(4).with_weights(np.ones(6, np.float32))
        g = G.disjoint_union([k4, c4], isolated=1)
        S = [1, 4, 6, 8]
    else:
        src = np.array([0, 0, 1, 1, 2, 3, 4, 2], dtype=np.int32)
        dst = np.array([1, 2, 2, 3, 4, 4, 5, 5], dtype=np.int32)
        g = G.EdgeList(6, src, dst, np.array([0.5, 2.0, 1.0, 4.0, 1.5, 0.75, 3.0, 1.0], np.float32))
        S = [0, 4]
    edges = [(int(min(a, b)), int(max(a, b))) for a, b in zip(g.src, g.dst)]
    edge_index = {e: i for i, e in enumerate(edges)}
    w = np.ones(g.m) if g.w is None else g.w.astype(np.float64)
    forests = _rooted_forests(g.n, edges, S)
    weight = np.array([np.prod(w[list(f)]) for f in forests])
    L = E.laplacian(E.adjacency(g.n, g.src, g.dst, g.w))
    keep = [i for i in range(g.n) if i not in S]
    assert weight.sum() == pytest.approx(np.linalg.det(L[np.ix_(keep, keep)]), rel=1e-9)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    nsamp = 30 * len(forests) + 2000
    r = W.fastwalk_sample(csr, S, 4321, 0, 0, nsamp, want_parents=True)
    assert (r["parents"][:, S] == -1).all()
    idx = {f: i for i, f in enumerate(forests)}
    counts = np.zeros(len(forests))
    for par in r["parents"]:
        f = frozenset(edge_index[(min(u, p), max(u, p))] for u, p in enumerate(par) if p >= 0)
        counts[idx[f]] += 1
    p = st.chisquare(counts, weight / weight.sum() * nsamp).pvalue
    assert p > 1e-3


def test_expected_departures_with_a_root_set():
    """E[departures from u in a forest rooted at S] = d_u (L_S^{-1})_uu (Lemma 5.2 with the
    walk trapped at a set), and the mean number of steps is their sum."""
    g = G.erdos_renyi_lcc(30, 4, 9)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 10))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    S = [2, 11, 23]
    l = 40000
    r = W.fastwalk_sample(csr, S, 2025, 0, 0, l, threads=4)
    t = E.grounded_inverse_diag_set(g.n, g.src, g.dst, g.w, S)
    mean = r["visits"].astype(float) / l
    var = r["visits_sq"].astype(float) / l - mean ** 2
    mask = ~np.isin(np.arange(g.n), S)
    z = (mean[mask] - t[mask]) / np.sqrt(var[mask] / l)
    assert np.max(np.abs(z)) < 5.0
    assert (r["visits"][S] == 0).all()
    s = r["steps"].astype(float)
    assert abs(s.mean() - t.sum()) < 5 * s.std() / np.sqrt(l)
    # one root given as a set is the rooted tree
    one = W.fastwalk_sample(csr, [csr.pivot], 5, 0, 0, 20, want_parents=True)
    ref = W.fastwalk_sample(csr, csr.pivot, 5, 0, 0, 20, want_parents=True)
    for key in ("visits", "visits_sq", "steps", "hash", "parents"):
        np.testing.assert_array_equal(one[key], ref[key])
    with pytest.raises(ValueError):
        W.fastwalk_sample(csr, [3, 3], 5, 0, 0, 2)


def test_expected_departures_on_a_disconnected_graph():
    """Three components (a weighted ER graph, a 4 x 4 grid, an isolated node) and a root set
    with one node in each (two in the grid): L_S is block diagonal and E[departures from u] =
    d_u (L_S^{-1})_uu holds component by component; the isolated root never departs."""
    er = G.erdos_renyi_lcc(24, 4, 19)
    er = er.with_weights(G.uniform_weights(er.m, 0.5, 2.0, 20))
    grid = G.grid_with_deletions(16, 0.0, 0).with_weights(np.ones(24, np.float32))
    g = G.disjoint_union([er, grid], isolated=1)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    S = [5, er.n + 3, er.n + 12, g.n - 1]
    l = 40000
    r = W.fastwalk_sample(csr, S, 77, 0, 0, l, threads=4)
    t = E.grounded_inverse_diag_set(g.n, g.src, g.dst, g.w, S)
    mean = r["visits"].astype(float) / l
    var = r["visits_sq"].astype(float) / l - mean ** 2
    mask = ~np.isin(np.arange(g.n), S)
    z = (mean[mask] - t[mask]) / np.sqrt(var[mask] / l)
    assert np.max(np.abs(z)) < 5.0
    assert (r["visits"][S] == 0).all()
    s = r["steps"].astype(float)
    assert abs(s.mean() - t.sum()) < 5 * s.std() / np.sqrt(l)


# ------------------------------------------------------------ trap walks ---------------
@pytest.mark.parametrize("case", ["er30_w", "K7", "C11"])
def test_trap_walk_visits_lemma_5_1(case):
    """Walks from u stopped at the trap v visit u (the start included) (calL_v^{-1})_uu times on
    average (Lemma 5.1); on K_n that is 2(n-1)/n, on C_n 2k(n-k)/n at distance k from v."""
    if case == "er30_w":
        g = G.erdos_renyi_lcc(30, 4, 9)
        g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 10))
    elif case == "K7":
        g = G.complete_graph(7)
    else:
        g = G.cycle_graph(11)
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    v = csr.pivot
    l = 20000
    r = W.trapwalk_sample(csr, v, 77, 0, 0, l, threads=4)
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    if case == "K7":
        np.testing.assert_allclose(np.delete(t, v), 2.0 * 6 / 7, rtol=1e-12)
    if case == "C11":
        k = np.minimum(np.abs(np.arange(11) - v), 11 - np.abs(np.arange(11) - v))
        np.testing.assert_allclose(np.delete(t, v), np.delete(2.0 * k * (11 - k) / 11, v), rtol=1e-12)
    mean = r["visits"].astype(float) / l
    var = r["visits_sq"].astype(float) / l - mean ** 2
    mask = np.arange(g.n) != v
    z = (mean[mask] - t[mask]) / np.sqrt(var[mask] / l)
    assert np.max(np.abs(z)) < 5.0
    assert r["visits"][v] == 0


def test_trap_walk_lengths_are_hitting_times():
    """The walks' total length over l walks per start node is l * sum_u H_uv (hitting times to
    the trap), checked against the spread of 40 independent walk ranges."""
    g = G.erdos_renyi_lcc(25, 4, 3)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 4))
    csr = W.OracleCSR(g.n, g.src, g.dst, g.w)
    v = csr.pivot
    h = E.hitting_times_to(g.n, g.src, g.dst, g.w, v)
    per = 500
    totals = np.array([W.trapwalk_sample(csr, v, 5, 0, c * per, per)["steps"] / per for c in range(40)])
    assert abs(totals.mean() - h.sum()) < 5 * totals.std(ddof=1) / np.sqrt(len(totals))


def test_trap_walk_range_and_thread_independence():
    g = G.barabasi_albert(60, 2, 8)
    csr = W.OracleCSR(g.n, g.src, g.dst, None)
    v = csr.pivot
    base = W.trapwalk_sample(csr, v, 3, 1, 0, 30)
    split = W.trapwalk_sample(csr, v, 3, 1, 0, 30, threads=4)
    a = W.trapwalk_sample(csr, v, 3, 1, 0, 13)
    b = W.trapwalk_sample(csr, v, 3, 1, 13, 17)
    for key in ("visits", "visits_sq"):
        np.testing.assert_array_equal(split[key], base[key])
        np.testing.assert_array_equal(a[key] + b[key], base[key])
    assert a["steps"] + b["steps"] == base["steps"] == split["steps"]
    assert not np.array_equal(W.trapwalk_sample(csr, v, 4, 1, 0, 30)["visits"], base["visits"])
