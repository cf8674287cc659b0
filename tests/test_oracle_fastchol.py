"""Pins of the FastChol oracle (Section 4, Algorithm 2) against the mathematics (no GPU).

IChol: with no dropping it is the exact Cholesky factor; with dropping it equals a dense
right-looking factorization written independently here (same drop rule, Schur updates in the
same order, so the same bits) and keeps the M-matrix signs, so its inverse is non-negative
(Lemma 4.3).  Sparse inverse: with a full window and no sparsification its columns are R^{-1}'s
and tau~ is the exact diag(calL_v^{-1}), so FastChol's RWC is the exact RWC; with sparsification
every column keeps a magnitude prefix whose dropped tail obeys the eps_p bound, is minimal,
and meets the relative bound of Theorem 4.4.
"""
import numpy as np
import pytest

import rwcgen as G
from oracle import exact as E
from oracle import fastchol as F


def _graph(name):
    if name == "er40_w":
        g = G.erdos_renyi_lcc(40, 4, 3)
        return g.with_weights(G.uniform_weights(g.m, 0.5, 2.0, 4))
    if name == "ba60":
        return G.barabasi_albert(60, 2, 5)
    if name == "grid36":
        return G.grid_with_deletions(36, 0.0, 1)
    if name == "star9":
        return G.star_graph(9)
    raise KeyError(name)


def _dense_lower(ptr, row, val):
    N = ptr.shape[0] - 1
    A = np.zeros((N, N))
    for j in range(N):
        for p in range(ptr[j], ptr[j + 1]):
            A[row[p], j] = val[p]
            A[j, row[p]] = val[p]
    return A


def _dense_factor(r_ptr, r_row, r_val):
    N = r_ptr.shape[0] - 1
    R = np.zeros((N, N))
    for j in range(N):
        for p in range(r_ptr[j], r_ptr[j + 1]):
            R[r_row[p], j] = r_val[p]
    return R


def _right_looking_ict(A, droptol):
    """Dense incomplete Cholesky, right-looking: column k is the pivot's square root and the
    scaled column below it, entries under droptol times the 1-norm of A's column dropped, then
    the trailing lower triangle loses the outer product of the kept column."""
    N = A.shape[0]
    S = np.tril(A).copy()
    R = np.zeros_like(A)
    norms = np.abs(np.tril(A)).sum(axis=0)
    for k in range(N):
        piv = np.sqrt(S[k, k])
        R[k, k] = piv
        for i in range(k + 1, N):
            x = S[i, k] / piv
            if x != 0.0 and abs(x) >= droptol * norms[k]:
                R[i, k] = x
        for j in range(k + 1, N):
            if R[j, k] == 0.0:
                continue
            for i in range(j, N):
                if R[i, k] != 0.0:
                    S[i, j] = S[i, j] - R[i, k] * R[j, k]
    return R


@pytest.mark.parametrize("name", ["er40_w", "ba60", "grid36", "star9"])
def test_ichol_without_dropping_is_cholesky(name):
    g = _graph(name)
    v = int(np.argmax(np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)))
    ptr, row, val, _ = F.grounded_normalized_lower(g.n, g.src, g.dst, g.w, v)
    A = _dense_lower(ptr, row, val)
    R = _dense_factor(*F.ichol(ptr, row, val, 0.0))
    np.testing.assert_allclose(R, np.linalg.cholesky(A), rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", ["er40_w", "ba60", "grid36"])
@pytest.mark.parametrize("droptol", [1e-4, 1e-2, 0.1])
def test_ichol_matches_dense_right_looking(name, droptol):
    g = _graph(name)
    v = int(np.argmax(np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)))
    ptr, row, val, _ = F.grounded_normalized_lower(g.n, g.src, g.dst, g.w, v)
    A = _dense_lower(ptr, row, val)
    r_ptr, r_row, r_val = F.ichol(ptr, row, val, droptol)
    R = _dense_factor(r_ptr, r_row, r_val)
    np.testing.assert_array_equal(R, _right_looking_ict(A, droptol))
    # M-matrix signs, the drop rule, and a non-negative inverse (Lemma 4.3)
    norms = np.abs(np.tril(A)).sum(axis=0)
    off = np.tril(R, -1)
    assert np.all(np.diag(R) > 0) and np.all(off <= 0)
    kept = off != 0
    assert np.all(np.abs(off)[kept] >= (droptol * norms[None, :].repeat(R.shape[0], 0))[kept])
    assert np.all(np.linalg.inv(R) >= -1e-13)
    if droptol >= 1e-2:
        assert r_ptr[-1] < np.count_nonzero(np.linalg.cholesky(A))   # something was dropped


@pytest.mark.parametrize("name", ["er40_w", "ba60", "grid36"])
def test_full_window_no_sparsification_is_exact(name):
    """w_s >= N and zeta >= N: S~ = R^{-1}; with exact Cholesky tau~ = diag(calL_v^{-1}) and the
    assembled RWC is the exact one (Theorem 3.1)."""
    g = _graph(name)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    v = int(np.argmax(deg))
    ptr, row, val, nodes = F.grounded_normalized_lower(g.n, g.src, g.dst, g.w, v)
    N = g.n - 1
    r_ptr, r_row, r_val = F.ichol(ptr, row, val, 0.02)
    R = _dense_factor(r_ptr, r_row, r_val)
    tau, s_ptr, s_row, s_val = F.sparse_inverse_columns(r_ptr, r_row, r_val, deg[nodes].astype(float), N, N, 0.0)
    Sinv = np.linalg.inv(R)
    S = np.zeros((N, N))
    for u in range(N):
        S[s_row[s_ptr[u]:s_ptr[u + 1]], u] = s_val[s_ptr[u]:s_ptr[u + 1]]
    np.testing.assert_allclose(S, Sinv, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(tau, (Sinv ** 2).sum(axis=0), rtol=1e-10)
    r = F.fastchol(g.n, g.src, g.dst, g.w, v, droptol=0.0, ws=N, zeta=N, eps_p=0.0)
    t = E.grounded_normalized_inverse_diag(g.n, g.src, g.dst, g.w, v)
    np.testing.assert_allclose(r["tau"], t, rtol=1e-9, atol=1e-12)
    rwc = E.apprwc(g.n, g.src, g.dst, g.w, v, r["tau"])
    np.testing.assert_allclose(rwc, E.rwc_by_hitting_times(g.n, g.src, g.dst, g.w), rtol=1e-8)


@pytest.mark.parametrize("eps_p,zeta", [(1e-3, 2), (1e-2, 0), (0.1, 4)])
def test_sparsified_columns_keep_a_bounded_prefix(eps_p, zeta):
    """Every column of S~ is the largest-magnitude prefix of S* (rebuilt from the definition out
    of the later columns of S~), its dropped tail has 1-norm <= eps_p ||S*||_1, one more dropped
    entry would break that, and ||S*||^2 - ||S~||^2 <= eps_p^2 n ||S*||^2 (Theorem 4.4)."""
    g = G.barabasi_albert(80, 3, 7)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n).astype(float)
    v = int(np.argmax(deg))
    ptr, row, val, nodes = F.grounded_normalized_lower(g.n, g.src, g.dst, g.w, v)
    N = g.n - 1
    r_ptr, r_row, r_val = F.ichol(ptr, row, val, 1e-4)
    R = _dense_factor(r_ptr, r_row, r_val)
    ws = 6.0
    tau, s_ptr, s_row, s_val = F.sparse_inverse_columns(r_ptr, r_row, r_val, deg[nodes], ws, zeta, eps_p)
    S = np.zeros((N, N))
    for u in range(N):
        S[s_row[s_ptr[u]:s_ptr[u + 1]], u] = s_val[s_ptr[u]:s_ptr[u + 1]]
    dmax = deg[nodes].max()
    dropped_any = False
    for u in range(N):
        w = min(int(np.floor(ws * (1 + deg[nodes][u] / dmax))), N)
        star = np.zeros(N)
        star[u] = 1.0 / R[u, u]
        for i in range(u + 1, min(u + w, N - 1) + 1):
            if R[i, u] != 0.0:
                star -= (R[i, u] / R[u, u]) * S[:, i]
        kept = S[:, u] != 0
        assert np.all(star[kept] == S[kept, u])                 # kept entries unchanged
        nz = np.count_nonzero(star)
        if nz <= zeta:
            assert np.count_nonzero(kept) == nz
            continue
        drop = (star != 0) & ~kept
        dropped_any |= bool(drop.any())
        if drop.any() and kept.any():
            assert np.abs(star[drop]).max() <= np.abs(star[kept]).min()
        l1 = np.abs(star).sum()
        tail = np.abs(star[drop]).sum()
        assert tail <= eps_p * l1 * (1 + 1e-12)
        if kept.any():
            assert tail + np.abs(star[kept]).min() > eps_p * l1 * (1 - 1e-12)   # minimal
        s2, t2 = (star ** 2).sum(), (S[:, u] ** 2).sum()
        assert abs(s2 - t2) <= eps_p ** 2 * N * s2 * (1 + 1e-9)
        assert tau[u] == pytest.approx(t2, rel=1e-12)
    assert dropped_any
    assert np.all(S >= 0)                                        # Lemma 4.3 survives truncation
