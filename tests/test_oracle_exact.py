"""Pins of the exact-RWC oracle against the mathematics (no GPU)."""
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import rwcgen as G
from oracle import exact as E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_graphs():
    er = G.erdos_renyi_lcc(40, 5, 11)
    ba = G.barabasi_albert(50, 2, 12)
    grid = G.grid_with_deletions(36, 0.1, 13)
    return [
        er,
        er.with_weights(G.uniform_weights(er.m, 0.5, 2.0, 21)),
        ba.with_weights(G.uniform_weights(ba.m, 1.0, 4.0, 22)),
        grid,
        G.path_graph(9),
    ]


@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: g.name)
def test_three_characterisations_agree(g):
    h_def = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    h_eq2 = E.rwc_normalized_pinv(g.n, g.src, g.dst, g.w)
    h_pinv = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w)
    np.testing.assert_allclose(h_eq2, h_def, rtol=1e-11)
    np.testing.assert_allclose(h_pinv, h_def, rtol=1e-11)
    # the Cholesky route used for the larger exact checks
    h_chol = E.rwc_laplacian_pinv_cholesky(g.n, g.src, g.dst, g.w)
    np.testing.assert_allclose(h_chol, h_def, rtol=1e-10)


def _closed_forms():
    rows = []
    with open(os.path.join(GOLDEN, "rwc_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, n, qty, val = [x.strip() for x in line.split("|")]
            rows.append((kind, int(n), qty, float(Fraction(val))))
    return rows


@pytest.mark.parametrize("kind,n,qty,val", _closed_forms())
def test_closed_forms(kind, n, qty, val):
    g = {"K": G.complete_graph, "S": G.star_graph, "C": G.cycle_graph}[kind](n)
    if qty == "steps":
        got = E.expected_steps_per_tree(g.n, g.src, g.dst, None, 0)
        assert got == pytest.approx(val, rel=1e-12)
        return
    for fn in (E.rwc_by_hitting_times, E.rwc_laplacian_pinv, E.rwc_normalized_pinv):
        h = fn(g.n, g.src, g.dst, None)
        if qty == "rwc_any":
            np.testing.assert_allclose(h, val, rtol=1e-12)
        elif qty == "rwc_centre":
            assert h[0] == pytest.approx(val, rel=1e-12)
        else:
            np.testing.assert_allclose(h[1:], val, rtol=1e-12)


@pytest.mark.parametrize("g", _small_graphs()[:3], ids=lambda g: g.name)
def test_kemeny_invariant(g):
    """sum_u pi_u H_u equals the trace of the normalised-Laplacian pseudo-inverse (Eq. (2)),
    i.e. Kemeny's constant, which networkx computes from the spectrum of P independently."""
    h = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    A = E.adjacency(g.n, g.src, g.dst, g.w)
    pi = A.sum(1) / A.sum()
    nxg = nx.Graph()
    nxg.add_nodes_from(range(g.n))
    ww = np.ones(g.m) if g.w is None else g.w
    nxg.add_weighted_edges_from(zip(g.src.tolist(), g.dst.tolist(), ww.tolist()))
    kem = nx.kemeny_constant(nxg, weight="weight")
    assert pi @ h == pytest.approx(kem, rel=1e-10)
    assert pi @ h == pytest.approx(E.kemeny_from_spectrum(g.n, g.src, g.dst, g.w), rel=1e-10)


@pytest.mark.parametrize("g", _small_graphs()[:3], ids=lambda g: g.name)
def test_theorem_3_1_every_pivot(g):
    """AppRWC (Algorithm 1) fed the exact diagonal of calL_v^{-1} and an exact solve returns
    the exact RWC for every choice of pivot (Theorem 3.1)."""
    h_def = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    for v in range(g.n):
        t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
        np.testing.assert_allclose(E.apprwc(g.n, g.src, g.dst, g.w, v, t), h_def, rtol=1e-10)


def test_apprwc_sparse_solvers_match_dense():
    g = _small_graphs()[2]
    v = E.pivot_of(g.n, g.src, g.dst, g.w)
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    dense = E.apprwc(g.n, g.src, g.dst, g.w, v, t, "dense")
    for m in ("sparse_direct", "sparse_cg"):
        np.testing.assert_allclose(E.apprwc(g.n, g.src, g.dst, g.w, v, t, m), dense, rtol=1e-10)


def test_apprwc_detects_a_dropped_term():
    """Plant a mistake in the oracle's assembly (drop the cross term of Eq. (3)) and check
    that the definition-based pin notices it."""
    g = _small_graphs()[1]
    v = 0
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    A = E.adjacency(g.n, g.src, g.dst, g.w)
    d = A.sum(1)
    vol = d.sum()
    y = E.laplacian_pinv(E.laplacian(A))  # only used to build a wrong variant below
    sd = np.sqrt(d)
    Pi = np.eye(g.n) - np.outer(sd, sd) / vol
    col = (Pi @ np.diag(sd) @ y @ np.diag(sd) @ Pi)[:, v]
    wrong = (t - (d / d[v]) * col[v]) / (d / vol)
    h_def = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    assert np.max(np.abs(wrong - h_def) / h_def) > 1e-3


def test_grounded_diagonal_is_degree_times_resistance():
    """(calL_v^{-1})_uu = d_u R_uv (proof of Theorem 3.1), R from networkx."""
    g = _small_graphs()[1]
    v = 3
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    d = E.adjacency(g.n, g.src, g.dst, g.w).sum(1)
    nxg = nx.Graph()
    nxg.add_weighted_edges_from(zip(g.src.tolist(), g.dst.tolist(), g.w.astype(float).tolist()))
    for u in [0, 1, 7, 20]:
        # invert_weight=False: networkx then uses the weight itself as the conductance
        r = nx.resistance_distance(nxg, u, v, weight="weight", invert_weight=False)
        assert t[u] == pytest.approx(d[u] * r, rel=1e-9)


def test_relabel_and_weight_scale_invariance():
    g = _small_graphs()[1]
    h = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w)
    perm = np.random.default_rng(5).permutation(g.n)
    hp = E.rwc_laplacian_pinv(g.n, perm[g.src], perm[g.dst], g.w)
    np.testing.assert_allclose(hp[perm], h, rtol=1e-11)
    hs = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w.astype(np.float64) * 3.0)
    np.testing.assert_allclose(hs, h, rtol=1e-11)


def test_pivot_hitting_assembly_identity():
    """For every pivot v: H_u = vol (calL_v^{-1})_uu / d_u - 2 H_uv + H_v, the form the GPU
    assembly uses (Eq. (3) with the pivot column written through hitting times)."""
    g = _small_graphs()[2]
    h_def = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    d = E.adjacency(g.n, g.src, g.dst, g.w).sum(1)
    vol = d.sum()
    for v in (0, 9, E.pivot_of(g.n, g.src, g.dst, g.w)):
        t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
        hv = E.hitting_times_to(g.n, g.src, g.dst, g.w, v)
        rv = d @ hv / vol
        assert rv == pytest.approx(h_def[v], rel=1e-11)
        f = vol * t / d - 2.0 * hv + rv
        f[v] = rv
        np.testing.assert_allclose(f, h_def, rtol=1e-10)


def test_error_measures():
    x = np.array([1.0, 2.0, 4.0])
    assert E.mean_relative_error(x, x * 1.1) == pytest.approx(0.1)
    assert E.kendall_tau_a(x, x) == 1.0
    assert E.kendall_tau_a(x, -x) == -1.0


def test_ba20k_fixture_matches_the_hitting_time_definition():
    """The stored exact RWC of BA(20 000, 5) (dense Cholesky route) against the definition
    H_u = sum_i pi_i H_iu, each H_.u from one sparse grounded solve (L_u h = d_{-u}), at 52
    of the stored nodes."""
    import scipy.sparse.linalg as spla
    rows = []
    with open(os.path.join(GOLDEN, "ba20k_exact_rwc.txt")) as f:
        for line in f:
            if not line.startswith("#"):
                u, val = line.split("|")
                rows.append((int(u), float(val)))
    assert len(rows) >= 2000
    g = G.barabasi_albert(20_000, 5, 1002)
    L, d = E._sparse_laplacian(g.n, g.src, g.dst, g.w)
    # the pivot, the first and last stored nodes and 50 more spread over the file
    picks = sorted(set([0, len(rows) - 1] + np.linspace(0, len(rows) - 1, 52).astype(int).tolist()))
    assert len(picks) >= 50
    for u, val in [rows[i] for i in picks]:
        keep = np.ones(g.n, dtype=bool)
        keep[u] = False
        Lu = L[keep][:, keep].tocsr()
        h, info = spla.cg(Lu, d[keep], rtol=1e-14, atol=0.0, maxiter=5000,
                          M=spla.LinearOperator(Lu.shape, matvec=lambda x: x / d[keep]))
        assert info == 0
        assert abs(d[keep] @ h / d.sum() - val) <= 1e-9 * val


def test_group_rwc_definition_and_marginal_formula():
    """Group RWC H_S (hitting time to a set, stationary start): one node is that node's RWC;
    the star's centre gives 1/2; adding a node u to S, the rank-one form H_S - d_u h_u^2 /
    (vol d_u (L_S^{-1})_uu) equals H_{S + u} computed from its own definition, for every u."""
    g = _small_graphs()[2]
    h_def = E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w)
    for v in (0, 5):
        assert E.group_rwc(g.n, g.src, g.dst, g.w, [v]) == pytest.approx(h_def[v], rel=1e-11)
    star = G.star_graph(9)
    assert E.group_rwc(star.n, star.src, star.dst, None, [0]) == pytest.approx(0.5, rel=1e-12)
    for S in ([0], [1, 6], [2, 3, 9]):
        t = E.grounded_inverse_diag_set(g.n, g.src, g.dst, g.w, S)
        est = E.group_marginal_estimate(g.n, g.src, g.dst, g.w, S, t)
        for u in range(g.n):
            want = E.group_rwc(g.n, g.src, g.dst, g.w, sorted(set(S) | {u}))
            assert est[u] == pytest.approx(want, rel=1e-9), (S, u)
    # a planted slip (dropping d_u) is caught
    t = E.grounded_inverse_diag_set(g.n, g.src, g.dst, g.w, [1, 6])
    d = E.adjacency(g.n, g.src, g.dst, g.w).sum(1)
    bad = E.group_marginal_estimate(g.n, g.src, g.dst, g.w, [1, 6], t * d)
    want = np.array([E.group_rwc(g.n, g.src, g.dst, g.w, sorted({1, 6, u})) for u in range(g.n)])
    assert np.max(np.abs(bad - want) / want) > 1e-3


def test_er1000_fixture_matches_the_definition():
    """The stored exact RWC of the ER(1000, 8) component (pseudo-inverse route) against the
    hitting-time definition at 40 nodes, each from its own grounded solve."""
    import scipy.sparse.linalg as spla
    rows = []
    with open(os.path.join(GOLDEN, "er1000_exact_rwc.txt")) as f:
        for line in f:
            if not line.startswith("#"):
                u, val = line.split("|")
                rows.append((int(u), float(val)))
    g = G.erdos_renyi_lcc(1000, 8, 1001)
    assert len(rows) == g.n
    L, d = E._sparse_laplacian(g.n, g.src, g.dst, g.w)
    for u, val in [rows[i] for i in np.linspace(0, g.n - 1, 40).astype(int)]:
        keep = np.ones(g.n, dtype=bool)
        keep[u] = False
        h = spla.spsolve(L[keep][:, keep].tocsc(), d[keep])
        assert abs(d[keep] @ h / d.sum() - val) <= 1e-9 * val
