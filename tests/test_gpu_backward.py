"""Parity of rwc_backward (the adjoint of sum_j g_j RWC_j) with the CPU gradient oracle.

The gradient is floating point: the solves stop at a relative residual `tol`, which bounds
the relative error of each L^+ y by cond(L_v) * tol; with tol = 1e-12 and the condition
numbers of these graphs (< 1e4) the assembled gradient agrees with the dense FP64 reference
to better than 1e-7 of its largest entry, the tolerance used below.
"""
import numpy as np
import pytest
import torch

import rwcgen as G
from oracle import gradient as GR

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _graph(n, m, seed):
    g = G.barabasi_albert(n, m, seed)
    return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, seed + 1))


def _targets(n, k, seed, signed=False):
    rng = np.random.default_rng(seed)
    t = rng.choice(n, size=k, replace=False).astype(np.int32)
    gv = rng.uniform(0.5, 2.0, size=k) if signed else np.ones(k)
    if signed:
        gv[::3] *= -1.0
    return t, gv


def _close(got, want, rel):
    scale = np.abs(want).max()
    assert np.max(np.abs(got - want)) <= rel * scale, (np.max(np.abs(got - want)) / scale)


@pytest.mark.parametrize("signed", [False, True])
def test_exact_mode_matches_dense_gradient(signed):
    g = _graph(2000, 4, 71)
    t, gv = _targets(g.n, 20, 3, signed)
    gd = np.zeros(g.n)
    gd[t] = gv
    want = GR.grad_exact(g.n, g.src, g.dst, g.w, gd)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    res = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=0, tol=1e-12)
    got = res["grad_w"].cpu().numpy()
    _close(got, want, 1e-7)
    assert abs(np.dot(g.w, got)) <= 1e-8 * np.abs(g.w * got).sum()


@pytest.mark.parametrize("signed", [False, True])
def test_sketch_mode_matches_oracle_probes(signed):
    g = _graph(600, 3, 81)
    t, gv = _targets(g.n, 15, 4, signed)
    gd = np.zeros(g.n)
    gd[t] = gv
    k, seed = 16, 12345
    cols = GR.probe_columns(g.n, t, gv, k, seed)
    want = GR.grad_from_probes(g.n, g.src, g.dst, g.w, gd, cols)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    got = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=k, seed=seed, tol=1e-12)["grad_w"].cpu().numpy()
    _close(got, want, 1e-7)
    # the sketch keeps Euler's identity for the scale-invariant RWC exactly
    assert abs(np.dot(g.w, got)) <= 1e-8 * np.abs(g.w * got).sum()


def test_autograd_function_uses_the_adjoint():
    g = _graph(800, 3, 91)
    t, gv = _targets(g.n, 10, 5)
    w = torch.tensor(g.w, device="cuda", requires_grad=True)
    rwc = P.RWCFunction.apply(w, g.n, g.src, g.dst, 64, 7)
    loss = rwc[torch.as_tensor(t, device="cuda", dtype=torch.int64)].sum()
    loss.backward()
    gd = np.zeros(g.n)
    gd[t] = 1.0
    want = GR.grad_exact(g.n, g.src, g.dst, g.w, gd)
    _close(w.grad.double().cpu().numpy(), want, 1e-5)   # float32 gradient


@pytest.mark.parametrize("k", [0, 64])
def test_ba100k_sampled_edges_match_sparse_oracle(k):
    """BA(1e5, 4), w ~ U[0.5, 2], 100 targets with g = 1: the GPU gradient at 20 sampled
    edges equals the oracle's sparse evaluation (exact, or with the same 64 probes)."""
    g = _graph(100_000, 4, 1004)
    t, gv = _targets(g.n, 100, 6)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    res = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=k, seed=2004, tol=1e-11)
    got = res["grad_w"].cpu().numpy()
    edges = np.random.default_rng(8).choice(g.m, size=20, replace=False)
    cols = None if k == 0 else GR.probe_columns(g.n, t, gv, k, 2004)
    want = GR.grad_at_edges_sparse(g.n, g.src, g.dst, g.w, t, gv, edges, cols)
    _close(got[edges], want, 1e-6)
    assert abs(np.dot(g.w, got)) <= 1e-7 * np.abs(g.w * got).sum()


def test_ba2000_gradient_against_central_differences_on_50_edges():
    """BA(2000, 4), w ~ U[0.5, 2], loss = sum of RWC over 100 targets: the GPU adjoint (exact
    probe mode) against central differences of the exact FP64 loss on 50 random edges, step
    h = 1e-4 w_e.  The perturbed losses are exact: w_e -> w_e + h changes L by h b b^T, so
    (L + J/n)^{-1} changes by the Sherman-Morrison rank-one term (checked against a full dense
    re-evaluation on two edges); the degrees of e's endpoints and vol change by h and 2h.  The
    quotient's truncation error is O(h^2), its rounding error ~1e-16 * loss / h."""
    from oracle import exact as E
    g = _graph(2000, 4, 91)
    t, gv = _targets(g.n, 100, 92)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    got = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=0, tol=1e-12)["grad_w"].cpu().numpy()

    w0 = g.w.astype(np.float64)
    n = g.n
    A = E.adjacency(n, g.src, g.dst, w0)
    d0 = A.sum(axis=1)
    Minv = np.linalg.inv(E.laplacian(A) + 1.0 / n)       # (L + J/n)^{-1}

    def loss_perturbed(e, h):
        a, b = int(g.src[e]), int(g.dst[e])
        u = Minv[:, a] - Minv[:, b]                        # M^{-1} b_e
        c = h / (1.0 + h * (u[a] - u[b]))
        d = d0.copy()
        d[a] += h
        d[b] += h
        vol = d.sum()
        diag_t = np.diag(Minv)[t] - c * u[t] ** 2 - 1.0 / n
        Ld = Minv @ d - c * u * (u @ d) - vol / n           # L'^+ d with L'^+ = M'^{-1} - J/n
        return float(np.dot(gv, vol * diag_t - 2.0 * Ld[t] + (d @ Ld) / vol))

    def loss_dense(w):
        return float(np.dot(gv, E.rwc_laplacian_pinv(n, g.src, g.dst, w)[t]))

    edges = np.random.default_rng(93).choice(g.m, size=50, replace=False)
    for e in edges[:2]:
        w1 = w0.copy()
        w1[e] += 1e-4 * w0[e]
        assert abs(loss_perturbed(e, 1e-4 * w0[e]) - loss_dense(w1)) <= 1e-11 * abs(loss_dense(w1))
    fd = []
    for e in edges:
        h = 1e-4 * w0[e]
        fd.append((loss_perturbed(e, h) - loss_perturbed(e, -h)) / (2.0 * h))
    _close(got[edges], np.array(fd), 1e-6)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_smallest_graphs_match_dense_gradient(n):
    """Paths of two to four nodes, every node a target (exact mode): the adjoint's SpMM cuts
    the CSR into a single segment, with no boundary for the fix-up to join.  With one edge the
    gradient is zero (RWC does not change when every weight is scaled, so w dl/dw = 0)."""
    g = G.path_graph(n)
    g = g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 40 + n))
    t = np.arange(n, dtype=np.int32)
    gv = np.linspace(1.0, 2.0, n)
    gd = np.zeros(n)
    gd[t] = gv
    want = GR.grad_exact(n, g.src, g.dst, g.w, gd)
    Gd = P.Graph(n, g.src, g.dst, g.w)
    got = P.backward(Gd, P.dense_g(n, t, gv, "cuda"), k=0, tol=1e-13)["grad_w"].cpu().numpy()
    if n == 2:
        assert abs(got[0]) <= 1e-12 and abs(want[0]) <= 1e-12
    else:
        _close(got, want, 1e-7)


def test_rows_spanning_many_segments_match_dense_gradient():
    """Two hubs joined by an edge, with 2400 and 1800 leaves: the SpMM's segments hold about
    64 units of work, so each hub row is cut by dozens of segment boundaries and summed by the
    fix-up over every segment it spans.  The second hub is not the pivot, so its cut row
    reaches the solution; targets on both hubs and on leaves of each."""
    a, b = 2400, 1800
    n = a + b + 2
    src = np.concatenate([[0], np.zeros(a, np.int64), np.ones(b, np.int64)])
    dst = np.concatenate([[1], 2 + np.arange(a), 2 + a + np.arange(b)])
    w = G.uniform_weights(len(src), 0.5, 2.0, 61)
    t = np.array([0, 1, 2, 3, a + 2, a + 3, n - 1], dtype=np.int32)
    gv = np.array([1.0, 2.0, 0.5, 1.5, 0.75, 1.25, 1.0])
    gd = np.zeros(n)
    gd[t] = gv
    want = GR.grad_exact(n, src, dst, w, gd)
    Gd = P.Graph(n, src, dst, w)
    got = P.backward(Gd, P.dense_g(n, t, gv, "cuda"), k=0, tol=1e-13)["grad_w"].cpu().numpy()
    _close(got, want, 1e-7)
    assert abs(np.dot(w, got)) <= 1e-8 * np.abs(w * got).sum()


def test_more_than_128_columns_match_dense_gradient():
    """Exact mode with 140 targets: 142 solve columns, so the SpMM runs a second pass over its
    segments for columns 128 .. 141 (a 14-column block of P)."""
    g = _graph(1500, 3, 71)
    t, gv = _targets(g.n, 140, 9, signed=True)
    gd = np.zeros(g.n)
    gd[t] = gv
    want = GR.grad_exact(g.n, g.src, g.dst, g.w, gd)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    got = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=0, tol=1e-12)["grad_w"].cpu().numpy()
    _close(got, want, 1e-7)


def test_two_full_column_blocks_match_oracle_probes():
    """Sketch mode with 63 probes per sign class and both classes present: 128 columns, two
    full 64-column blocks of P and no remainder."""
    g = _graph(700, 3, 83)
    t, gv = _targets(g.n, 30, 10, signed=True)
    gd = np.zeros(g.n)
    gd[t] = gv
    k, seed = 63, 777
    cols = GR.probe_columns(g.n, t, gv, k, seed)
    want = GR.grad_from_probes(g.n, g.src, g.dst, g.w, gd, cols)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    got = P.backward(Gd, P.dense_g(g.n, t, gv, "cuda"), k=k, seed=seed, tol=1e-12)["grad_w"].cpu().numpy()
    _close(got, want, 1e-7)


def test_iterations_past_convergence_change_nothing():
    """The host looks at the columns' convergence every `check_every` iterations; the ones
    launched past the last column's convergence return at once.  Looking after every
    iteration, every 7 or every 16 gives the same iteration count (the one run) and the same
    gradient bit for bit."""
    g = _graph(2000, 4, 75)
    t, gv = _targets(g.n, 12, 11, signed=True)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    gd = P.dense_g(g.n, t, gv, "cuda")
    runs = [P.backward(Gd, gd, k=16, seed=5, tol=1e-10, check_every=c) for c in (1, 7, 16)]
    iters = [r["iters"] for r in runs]
    assert iters[0] == iters[1] == iters[2], iters
    for r in runs[1:]:
        assert torch.equal(r["grad_w"], runs[0]["grad_w"])
