"""Pins of the gradient oracle: the 5-term adjoint formula against reverse-mode autodiff of a
different RWC formula, central finite differences, homogeneity, and the sketch's statistics."""
import numpy as np
import pytest

import rwcgen as G
from oracle import gradient as GR


def _graphs():
    er = G.erdos_renyi_lcc(40, 5, 31)
    ba = G.barabasi_albert(60, 3, 32)
    return [er.with_weights(G.uniform_weights(er.m, 0.5, 2.0, 41)),
            ba.with_weights(G.uniform_weights(ba.m, 0.5, 2.0, 42))]


def _targets(n, k, seed):
    g = np.zeros(n)
    g[np.random.default_rng(seed).choice(n, size=k, replace=False)] = 1.0
    return g


@pytest.mark.parametrize("gr", _graphs(), ids=lambda g: g.name)
def test_formula_matches_autograd(gr):
    g = _targets(gr.n, 6, 1)
    np.testing.assert_allclose(GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g),
                               GR.grad_autograd(gr.n, gr.src, gr.dst, gr.w, g), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("gr", _graphs(), ids=lambda g: g.name)
def test_formula_matches_finite_differences(gr):
    g = np.random.default_rng(3).uniform(0.0, 2.0, size=gr.n)   # signed targets are fine here
    grad = GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g)
    w = gr.w.astype(np.float64)
    for e in np.random.default_rng(4).choice(gr.m, size=8, replace=False):
        h = 1e-5 * w[e]
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (GR.loss(gr.n, gr.src, gr.dst, wp, g) - GR.loss(gr.n, gr.src, gr.dst, wm, g)) / (2 * h)
        assert grad[e] == pytest.approx(fd, rel=1e-6, abs=1e-7)


@pytest.mark.parametrize("gr", _graphs(), ids=lambda g: g.name)
def test_homogeneity(gr):
    """RWC is invariant under w -> c w, so sum_e w_e dl/dw_e = 0 (Euler)."""
    g = _targets(gr.n, 5, 2)
    grad = GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g)
    scale = np.abs(gr.w * grad).sum()
    assert abs(np.dot(gr.w, grad)) < 1e-11 * scale


def test_sketch_exact_mode_equals_formula():
    gr = _graphs()[0]
    g = _targets(gr.n, 7, 5)
    supp = np.flatnonzero(g)
    R = np.zeros((supp.size, gr.n))
    R[np.arange(supp.size), supp] = np.sqrt(supp.size)
    np.testing.assert_allclose(GR.grad_sketch(gr.n, gr.src, gr.dst, gr.w, g, R),
                               GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g), rtol=1e-10, atol=1e-12)


def test_sketch_unbiased_homogeneous_and_variance():
    gr = _graphs()[1]
    g = _targets(gr.n, 10, 6)
    exact = GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g)
    rng = np.random.default_rng(9)
    k, reps = 8, 3000
    draws = np.empty((reps, gr.m))
    for r in range(reps):
        R = rng.choice([-1.0, 1.0], size=(k, gr.n))
        draws[r] = GR.grad_sketch(gr.n, gr.src, gr.dst, gr.w, g, R)
        if r < 5:   # the sketch keeps sum_e w_e dl/dw_e = 0 exactly
            assert abs(np.dot(gr.w, draws[r])) < 1e-10 * np.abs(gr.w * draws[r]).sum()
    mean = draws.mean(axis=0)
    se = draws.std(axis=0) / np.sqrt(reps)
    assert np.max(np.abs(mean - exact) / (se + 1e-12)) < 5.0
    # Var(Q^_e) = (2/k)(|y|^4 - sum y_j^4) with y = G^{1/2} L^+ b_e for Rademacher probes;
    # the gradient's only random terms are -vol Q^_e + 2 trGL^, so check Q^ through a
    # fresh set of draws of Q^ alone for one edge.
    from oracle.exact import adjacency, laplacian, laplacian_pinv
    Lp = laplacian_pinv(laplacian(adjacency(gr.n, gr.src, gr.dst, gr.w)))
    e = 3
    a, b = int(gr.src[e]), int(gr.dst[e])
    y = np.sqrt(g) * (Lp[:, a] - Lp[:, b])
    qs = []
    for _ in range(20000):
        R = rng.choice([-1.0, 1.0], size=(k, gr.n))
        qs.append(np.mean((R @ y) ** 2))
    var_theory = 2.0 / k * ((y @ y) ** 2 - np.sum(y ** 4))
    assert np.var(qs) == pytest.approx(var_theory, rel=0.06)
    assert np.mean(qs) == pytest.approx(y @ y, rel=0.01)


# ---------------------------------------------------------------------------------------
# Pins of the probe-column helpers (probe_columns, grad_from_probes, grad_at_edges_sparse):
# they are the reference of the adjoint's GPU tests, so they are fixed here against the
# dense formula (itself pinned above by autograd, finite differences and homogeneity).
# ---------------------------------------------------------------------------------------
def _signed_targets(n, k, seed):
    """k targets with g of both signs (every third value negated)."""
    rng = np.random.default_rng(seed)
    t = rng.choice(n, size=k, replace=False).astype(np.int32)
    gv = rng.uniform(0.5, 2.0, size=k)
    gv[::3] *= -1.0
    return t, gv


def _dense(n, t, gv):
    g = np.zeros(n)
    g[t] = gv
    return g


@pytest.mark.parametrize("signed", [False, True])
@pytest.mark.parametrize("gi", [0, 1])
def test_exact_probe_columns_reproduce_the_formula(signed, gi):
    """k = 0: one column sqrt|g_j| e_j with coefficient sign(g_j) per target gives
    Q_e = sum_j g_j (L^+ b_e)_j^2 and trGL = sum_j g_j L^+_jj exactly."""
    gr = _graphs()[gi]
    t, gv = _signed_targets(gr.n, 9, 11 + gi)
    if not signed:
        gv = np.abs(gv)
    g = _dense(gr.n, t, gv)
    cols = GR.probe_columns(gr.n, t, gv, 0, 0)
    assert len(cols) == t.size
    np.testing.assert_allclose(GR.grad_from_probes(gr.n, gr.src, gr.dst, gr.w, g, cols),
                               GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g), rtol=1e-10, atol=1e-10)


def test_probe_columns_layout_and_signs():
    """Sketch columns: k per sign class present, positive class first, coefficients +1/k and
    -1/k, each probe supported on the targets of its class with entries +-sqrt|g|, and the
    Rademacher signs roughly balanced."""
    n = 50
    t, gv = _signed_targets(n, 12, 5)
    k = 7
    cols = GR.probe_columns(n, t, gv, k, 99)
    assert len(cols) == 2 * k
    pos, neg = t[gv > 0], t[gv < 0]
    signs = []
    for i, (c, y) in enumerate(cols):
        cls_targets = pos if i < k else neg
        assert c == pytest.approx((1.0 if i < k else -1.0) / k)
        assert set(np.flatnonzero(y)) == set(cls_targets.tolist())
        np.testing.assert_allclose(np.abs(y[t]), np.where(np.isin(t, cls_targets), np.sqrt(np.abs(gv)), 0.0))
        signs.extend(np.sign(y[cls_targets]).tolist())
    assert abs(np.mean(signs)) < 0.35
    # only one class present: k columns, all with +1/k
    cols_pos = GR.probe_columns(n, t, np.abs(gv), k, 99)
    assert len(cols_pos) == k and all(c == pytest.approx(1.0 / k) for c, _ in cols_pos)
    # another seed draws other signs
    other = GR.probe_columns(n, t, gv, k, 100)
    assert any(not np.array_equal(a[1], b[1]) for a, b in zip(cols, other))


def test_signed_two_class_sketch_is_unbiased_and_keeps_euler():
    """Signed g: the sketch with k probes per sign class, averaged over 2000 probe seeds,
    matches the exact gradient within 5 standard errors at every edge, and every single draw
    keeps sum_e w_e dl/dw_e = 0 (the sketch enters only through -vol Q^_e + 2 trGL^)."""
    gr = _graphs()[1]
    t, gv = _signed_targets(gr.n, 10, 21)
    g = _dense(gr.n, t, gv)
    exact = GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g)
    from oracle.exact import adjacency, laplacian, laplacian_pinv
    Lp = laplacian_pinv(laplacian(adjacency(gr.n, gr.src, gr.dst, gr.w)))
    a, b = gr.src.astype(np.int64), gr.dst.astype(np.int64)
    d = adjacency(gr.n, gr.src, gr.dst, gr.w).sum(1)
    vol = d.sum()
    base = exact + vol * (g[None, :] @ ((Lp[:, a] - Lp[:, b]) ** 2)).ravel() - 2.0 * float(g @ np.diag(Lp))
    k, reps = 4, 2000
    draws = np.empty((reps, gr.m))
    for r in range(reps):
        cols = GR.probe_columns(gr.n, t, gv, k, 1000 + r)
        # the sketched Q^ and trGL^ assembled from the probe columns, plugged into the
        # formula's deterministic part (same arithmetic as grad_from_probes, without
        # recomputing L^+ for every draw)
        Q = np.zeros(gr.m)
        tr = 0.0
        for c, y in cols:
            z = Lp @ y
            dz = z[a] - z[b]
            Q += c * dz * dz
            tr += c * float(y @ z)
        draws[r] = base - vol * Q + 2.0 * tr
        if r < 3:
            full = GR.grad_from_probes(gr.n, gr.src, gr.dst, gr.w, g, cols)
            np.testing.assert_allclose(full, draws[r], rtol=1e-9, atol=1e-9)
            assert abs(np.dot(gr.w, full)) < 1e-10 * np.abs(gr.w * full).sum()
    mean = draws.mean(axis=0)
    se = draws.std(axis=0, ddof=1) / np.sqrt(reps)
    assert np.max(np.abs(mean - exact) / (se + 1e-12)) < 5.0
    # a planted slip (the negative class with +1/k) is biased and caught by the same test
    slip = draws + 0.0
    for r in range(reps):
        cols = GR.probe_columns(gr.n, t, gv, k, 1000 + r)
        corr = 0.0
        Qc = np.zeros(gr.m)
        for c, y in cols:
            if c < 0:
                z = Lp @ y
                dz = z[a] - z[b]
                Qc += 2.0 * (-c) * dz * dz
                corr += 2.0 * (-c) * float(y @ z)
        slip[r] = draws[r] - vol * Qc + 2.0 * corr
    se_s = slip.std(axis=0, ddof=1) / np.sqrt(reps)
    assert np.max(np.abs(slip.mean(axis=0) - exact) / (se_s + 1e-12)) > 5.0


@pytest.mark.parametrize("signed", [False, True])
def test_sparse_evaluation_equals_dense(signed):
    """grad_at_edges_sparse (sparse grounded CG solves) equals the dense evaluation at sampled
    edges: exactly with cols=None, and from the same probe columns when they are given."""
    g0 = G.barabasi_albert(180, 3, 61)
    gr = g0.with_weights(G.uniform_weights(g0.m, 0.5, 2.0, 62))
    t, gv = _signed_targets(gr.n, 12, 23)
    if not signed:
        gv = np.abs(gv)
    g = _dense(gr.n, t, gv)
    edges = np.random.default_rng(5).choice(gr.m, size=25, replace=False)
    exact = GR.grad_exact(gr.n, gr.src, gr.dst, gr.w, g)
    scale = np.abs(exact).max()
    sp_exact = GR.grad_at_edges_sparse(gr.n, gr.src, gr.dst, gr.w, t, gv, edges)
    assert np.max(np.abs(sp_exact - exact[edges])) <= 1e-8 * scale
    cols = GR.probe_columns(gr.n, t, gv, 8, 4242)
    dense_probe = GR.grad_from_probes(gr.n, gr.src, gr.dst, gr.w, g, cols)
    sp_probe = GR.grad_at_edges_sparse(gr.n, gr.src, gr.dst, gr.w, t, gv, edges, cols=cols)
    assert np.max(np.abs(sp_probe - dense_probe[edges])) <= 1e-8 * np.abs(dense_probe).max()
    # the sketch is a different number from the exact value (so the two checks are distinct)
    assert np.max(np.abs(dense_probe - exact)) > 1e-3 * scale
