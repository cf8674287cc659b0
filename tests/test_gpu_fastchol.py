"""FastChol (Section 4, Algorithm 2) on the GPU against the oracle.

The GPU runs the serial algorithm's floating-point operations in the serial order (each entry's
updates in ascending column, in the left-looking chain and in the dense right-looking form alike;
norms and tails summed one entry at a time; the same total orders for sorting), so tau~, the
factor's size and S~'s size must equal the oracle's exactly, for both IChol methods.  With no
dropping, a full window and no sparsification tau~ is diag(calL_v^{-1}) and RWC is exact.
"""
import numpy as np
import pytest
import torch

import rwcgen as G
from oracle import exact as E
from oracle import fastchol as F

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2510_20604_amd")


def _graph(name):
    if name == "er300":
        return G.erdos_renyi_lcc(300, 5, 9)
    if name == "er1000_w":
        g = G.erdos_renyi_lcc(1000, 8, 1001)
        return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 3))
    if name == "ba2000":
        return G.barabasi_albert(2000, 3, 5)
    if name == "grid":
        return G.grid_with_deletions(900, 0.1, 7)
    if name == "path":
        return G.path_graph(130)
    if name == "star":
        return G.star_graph(50)
    raise KeyError(name)


def _oracle(g, v, droptol, ws, zeta, eps_p):
    d = np.zeros(g.n)
    w = np.ones(g.m) if g.w is None else g.w.astype(np.float64)
    np.add.at(d, g.src, w)
    np.add.at(d, g.dst, w)
    ptr, row, val, nodes = F.grounded_normalized_lower(g.n, g.src, g.dst, g.w, v)
    r_ptr, r_row, r_val = F.ichol(ptr, row, val, droptol)
    tau_c, snz = F.sparse_inverse(r_ptr, r_row, r_val, d[nodes], ws, zeta, eps_p)
    tau = np.zeros(g.n)
    tau[nodes] = tau_c
    return tau, int(r_ptr[-1]), int(snz.sum())


PARAMS = [(1e-4, 16.0, 16, 1e-3), (0.05, 4.0, 2, 0.05), (1e-3, 2.0, 0, 0.02)]


@pytest.mark.parametrize("method", ["chain", "dense"])
@pytest.mark.parametrize("params", PARAMS)
@pytest.mark.parametrize("name", ["er300", "er1000_w", "ba2000", "grid", "path", "star"])
def test_fastchol_matches_oracle_bit_for_bit(name, params, method):
    g = _graph(name)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    tau, fnz, snz = _oracle(g, Gd.pivot, *params)
    droptol, ws, zeta, eps_p = params
    r = P.fastchol(Gd, droptol=droptol, window=ws, zeta=zeta, eps_p=eps_p, factor_capacity=fnz + 16,
                   inverse_capacity=snz + 16, method=method)
    assert r["factor_entries"] == fnz
    assert r["inverse_entries"] == snz
    np.testing.assert_array_equal(r["tau"].cpu().numpy(), tau)


def test_dense_matches_oracle_on_ba20k():
    """The bench's BA(20000, 5) with its parameters: the dense form (the default at this size,
    19 999 launches, columns of up to thousands of kept entries spread over 255 workgroups)
    against the oracle, bit for bit."""
    g = G.barabasi_albert(20000, 5, 1002)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    lg = 15
    tau, fnz, snz = _oracle(g, Gd.pivot, 1e-4, float(lg), lg, 1e-3)
    r = P.fastchol(Gd, droptol=1e-4, window=float(lg), zeta=lg, eps_p=1e-3, method="dense")
    assert r["factor_entries"] == fnz
    assert r["inverse_entries"] == snz
    np.testing.assert_array_equal(r["tau"].cpu().numpy(), tau)


@pytest.mark.parametrize("method", ["chain", "dense"])
@pytest.mark.parametrize("name", ["er300", "grid", "ba2000"])
def test_exact_fastchol_gives_exact_rwc(name, method):
    """No dropping, a full window, no sparsification: tau~ = diag(calL_v^{-1}) and the assembled
    RWC (rwc_estimate_diag) is the exact RWC, with either factor."""
    g = _graph(name)
    if g.n > 1000:
        pytest.skip("dense inverse too large for this check")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    N = g.n - 1
    tri = N * (N + 1) // 2
    r = P.fastchol(Gd, droptol=0.0, window=float(N), zeta=N, eps_p=0.0, factor_capacity=tri, inverse_capacity=tri,
                   method=method)
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, Gd.pivot)
    np.testing.assert_allclose(r["tau"].cpu().numpy(), t, rtol=1e-9, atol=1e-12)
    rwc = P.estimate_diag(Gd, r["tau"])["rwc"].cpu().numpy()
    np.testing.assert_allclose(rwc, E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w), rtol=1e-8)


@pytest.mark.parametrize("method", ["chain", "dense"])
@pytest.mark.parametrize("name", ["er1000_w", "grid"])
def test_estimate_diag_matches_oracle_assembly(name, method):
    g = _graph(name)
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    r = P.fastchol(Gd, method=method)
    tau = r["tau"].cpu().numpy()
    got = P.estimate_diag(Gd, r["tau"])["rwc"].cpu().numpy()
    want = E.apprwc(g.n, g.src, g.dst, g.w, Gd.pivot, tau)
    np.testing.assert_allclose(got, want, rtol=1e-9)


def test_small_pools_are_reported():
    g = _graph("ba2000")
    Gd = P.Graph(g.n, g.src, g.dst, g.w)
    with pytest.raises(P.RWCError) as ei:
        P.fastchol(Gd, factor_capacity=g.n - 1)
    assert ei.value.status == -7
    with pytest.raises(P.RWCError) as ei:
        P.fastchol(Gd, inverse_capacity=10)
    assert ei.value.status == -7
    with pytest.raises(P.RWCError) as ei:
        P.fastchol(Gd, factor_capacity=g.n - 1, method="chain")
    assert ei.value.status == -7
    with pytest.raises(P.RWCError) as ei:
        P.fastchol(Gd, window=0.5)
    assert ei.value.status == -1


@pytest.mark.parametrize("method", ["chain", "dense"])
@pytest.mark.parametrize("n", [2, 3, 4])
def test_fastchol_on_the_smallest_graphs(n, method):
    """One, two and three columns (a single edge, the 3- and 4-node paths): the first launch is
    also the last column, the staging and the inverse's schedule hold one entry; and the 3-node
    star, whose pivot is the centre, leaves two columns without any off-diagonal entry."""
    for g in (G.path_graph(n), G.star_graph(n)) if n == 3 else (G.path_graph(n),):
        Gd = P.Graph(g.n, g.src, g.dst, g.w)
        tau, fnz, snz = _oracle(g, Gd.pivot, 1e-4, 2.0, 1, 1e-3)
        r = P.fastchol(Gd, droptol=1e-4, window=2.0, zeta=1, eps_p=1e-3, method=method)
        assert r["factor_entries"] == fnz
        assert r["inverse_entries"] == snz
        np.testing.assert_array_equal(r["tau"].cpu().numpy(), tau)
        assert tau[Gd.pivot] == 0.0
