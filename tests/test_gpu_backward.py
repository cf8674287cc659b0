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
    res = P.backward(Gd, t, gv, k=0, tol=1e-12)
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
    got = P.backward(Gd, t, gv, k=k, seed=seed, tol=1e-12)["grad_w"].cpu().numpy()
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
    res = P.backward(Gd, t, gv, k=k, seed=2004, tol=1e-11)
    got = res["grad_w"].cpu().numpy()
    edges = np.random.default_rng(8).choice(g.m, size=20, replace=False)
    cols = None if k == 0 else GR.probe_columns(g.n, t, gv, k, 2004)
    want = GR.grad_at_edges_sparse(g.n, g.src, g.dst, g.w, t, gv, edges, cols)
    _close(got[edges], want, 1e-6)
    assert abs(np.dot(g.w, got)) <= 1e-7 * np.abs(g.w * got).sum()
