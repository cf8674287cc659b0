"""Exact FP64 random walk centrality and the AppRWC assembly (CPU oracle, test-only).

Notation follows the paper.  For weighted graphs the adjacency holds the edge weights,
d is the weighted degree (strength), vol = sum(d) plays the role of 2m, P = D^{-1} A,
L = D - A and the normalised Laplacian is D^{-1/2} L D^{-1/2}.

All functions use dense matrices and are meant for n up to a few thousand (the
hitting-time definition for n up to ~100).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------------------
# Matrices (Section 2.2)
# ---------------------------------------------------------------------------------------
def adjacency(n: int, src, dst, w=None) -> np.ndarray:
    """Dense symmetric adjacency A with A_ij = w_ij (1 for unweighted graphs), Section 2.2."""
    A = np.zeros((n, n), dtype=np.float64)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    ww = np.ones(src.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    np.add.at(A, (src, dst), ww)
    np.add.at(A, (dst, src), ww)
    return A


def laplacian(A: np.ndarray) -> np.ndarray:
    """L = D - A (Section 2.2)."""
    return np.diag(A.sum(axis=1)) - A


def laplacian_pinv(L: np.ndarray) -> np.ndarray:
    """Moore-Penrose pseudo-inverse of a connected graph's Laplacian by the closed form
    L^+ = (L + J/n)^{-1} - J/n stated in Section 2.2."""
    n = L.shape[0]
    J = np.full((n, n), 1.0 / n)
    return np.linalg.inv(L + J) - J


# ---------------------------------------------------------------------------------------
# Three characterisations of RWC (Section 2.3)
# ---------------------------------------------------------------------------------------
def rwc_by_hitting_times(n: int, src, dst, w=None) -> np.ndarray:
    """The definition of Section 2.3: H_u = sum_i pi_i H_iu with pi = d / vol (Eq. (1)).

    H_iu, the expected first-passage time from i to u, solves the first-step equations
    H_iu = 1 + sum_k P_ik H_ku for i != u, H_uu = 0; one dense solve per target u.
    """
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    P = A / d[:, None]
    pi = d / d.sum()
    H = np.zeros(n)
    for u in range(n):
        idx = np.array([i for i in range(n) if i != u], dtype=np.int64)
        M = np.eye(n - 1) - P[np.ix_(idx, idx)]
        h = np.linalg.solve(M, np.ones(n - 1))
        H[u] = pi[idx] @ h
    return H


def rwc_normalized_pinv(n: int, src, dst, w=None) -> np.ndarray:
    """Eq. (2): H_u = (calL^+)_uu / pi_u, with calL^+ the pseudo-inverse of the normalised
    Laplacian computed by a symmetric eigendecomposition (numpy.linalg.pinv)."""
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    s = 1.0 / np.sqrt(d)
    Ln = s[:, None] * laplacian(A) * s[None, :]
    Lnp = np.linalg.pinv(Ln, hermitian=True)
    return np.diag(Lnp) / (d / d.sum())


def rwc_laplacian_pinv(n: int, src, dst, w=None) -> np.ndarray:
    """RWC from the unnormalised pseudo-inverse: H_u = vol L^+_uu - 2 (L^+ d)_u + d^T L^+ d / vol.

    Obtained from Eq. (2) by substituting the identity of Section 3 that relates the two
    pseudo-inverses, calL^+ = Pi D^{1/2} L^+ D^{1/2} Pi with Pi = I - D^{1/2} 1 1^T D^{1/2} / vol,
    and L^+ from the closed form of Section 2.2.
    """
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    vol = d.sum()
    Lp = laplacian_pinv(laplacian(A))
    Ld = Lp @ d
    return vol * np.diag(Lp) - 2.0 * Ld + (d @ Ld) / vol


def rwc_laplacian_pinv_cholesky(n: int, src, dst, w=None) -> np.ndarray:
    """The same formula as rwc_laplacian_pinv for larger n (tens of thousands of nodes):
    M = L + J/n is symmetric positive definite, so with M = C C^T (Cholesky) the diagonal of
    M^{-1} is the column sums of squares of C^{-1}, and L^+ = M^{-1} - J/n gives
    L^+_uu = (M^{-1})_uu - 1/n and L^+ d = M^{-1} d - (sum d / n) 1."""
    import scipy.linalg as sla
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    vol = d.sum()
    M = laplacian(A)
    del A
    M += 1.0 / n
    C = sla.cholesky(M, lower=True, overwrite_a=True, check_finite=False)
    Ci, info = sla.lapack.dtrtri(C, lower=1, overwrite_c=1)
    if info != 0:
        raise np.linalg.LinAlgError(f"dtrtri failed ({info})")
    diag = np.einsum("ij,ij->j", Ci, Ci) - 1.0 / n
    Md = Ci.T @ (Ci @ d)
    Ld = Md - vol / n
    return vol * diag - 2.0 * Ld + (d @ Ld) / vol


def kemeny_from_spectrum(n: int, src, dst, w=None) -> float:
    """Trace of calL^+ = sum over the non-zero eigenvalues of calL of 1 / lambda."""
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    s = 1.0 / np.sqrt(d)
    lam = np.linalg.eigvalsh(s[:, None] * laplacian(A) * s[None, :])
    return float(np.sum(1.0 / lam[1:]))


# ---------------------------------------------------------------------------------------
# Pivot quantities (Section 3, Lemma 5.1, Theorem 5.7)
# ---------------------------------------------------------------------------------------
def pivot_of(n: int, src, dst, w=None) -> int:
    """The pivot of Section 6.1 (the node of largest degree); ties go to the smallest id."""
    d = adjacency(n, src, dst, w).sum(axis=1)
    return int(np.flatnonzero(d == d.max())[0])


def grounded_normalized_inverse_diag(n: int, src, dst, w, v: int) -> np.ndarray:
    """(calL_v^{-1})_uu for u != v (entry v set to 0): the expected visits of a walk trapped
    at v, Lemma 5.1; also d_u times the effective resistance R_uv (proof of Theorem 3.1)."""
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    s = 1.0 / np.sqrt(d)
    Ln = s[:, None] * laplacian(A) * s[None, :]
    idx = np.array([i for i in range(n) if i != v], dtype=np.int64)
    inv = np.linalg.inv(Ln[np.ix_(idx, idx)])
    out = np.zeros(n)
    out[idx] = np.diag(inv)
    return out


def expected_steps_per_tree(n: int, src, dst, w, v: int) -> float:
    """Tr((I - P_v)^{-1}), the expected number of RandomNeighbor calls per rooted tree
    (Theorem 5.7)."""
    A = adjacency(n, src, dst, w)
    P = A / A.sum(axis=1)[:, None]
    idx = np.array([i for i in range(n) if i != v], dtype=np.int64)
    return float(np.trace(np.linalg.inv(np.eye(n - 1) - P[np.ix_(idx, idx)])))


def hitting_times_to(n: int, src, dst, w, v: int) -> np.ndarray:
    """h_u = H_uv, the hitting time from u to the pivot v: L_v h = d_{-v}, h_v = 0
    (first-step equations of Section 2.3 multiplied by D)."""
    A = adjacency(n, src, dst, w)
    d = A.sum(axis=1)
    L = laplacian(A)
    idx = np.array([i for i in range(n) if i != v], dtype=np.int64)
    h = np.zeros(n)
    h[idx] = np.linalg.solve(L[np.ix_(idx, idx)], d[idx])
    return h


# ---------------------------------------------------------------------------------------
# Algorithm 1 (AppRWC) with an exact Laplacian solve
# ---------------------------------------------------------------------------------------
def _sparse_laplacian(n: int, src, dst, w):
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    ww = np.ones(src.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    A = sp.coo_matrix((np.concatenate([ww, ww]), (np.concatenate([src, dst]),
                                                  np.concatenate([dst, src]))), shape=(n, n)).tocsr()
    d = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(d) - A).tocsr(), d


def lap_solve(n: int, src, dst, w, b: np.ndarray, method: str = "dense", v: int | None = None,
              rtol: float = 1e-14) -> np.ndarray:
    """LapSolve of Lemma 3.3 taken exact: a solution z of L z = b for b orthogonal to 1.

    ``dense`` returns L^+ b from the closed form.  ``sparse_direct`` / ``sparse_cg`` ground
    one node (row and column v removed, z_v = 0) and solve the remaining SPD system with
    SciPy's sparse LU or conjugate gradients; the result differs from L^+ b by a multiple
    of the all-ones vector, which every later step of Algorithm 1 projects away.  ``rtol``
    is the relative residual at which ``sparse_cg`` stops.
    """
    if method == "dense":
        return laplacian_pinv(laplacian(adjacency(n, src, dst, w))) @ b
    L, _ = _sparse_laplacian(n, src, dst, w)
    g = 0 if v is None else v
    keep = np.ones(n, dtype=bool)
    keep[g] = False
    Lg = L[keep][:, keep].tocsc()
    z = np.zeros(n)
    if method == "sparse_direct":
        z[keep] = spla.spsolve(Lg, b[keep])
    elif method == "sparse_cg":
        dg = Lg.diagonal()
        M = sp.diags(1.0 / dg)
        sol, info = spla.cg(Lg, b[keep], rtol=rtol, atol=0.0, maxiter=200000, M=M)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
        z[keep] = sol
    else:
        raise ValueError(method)
    return z


def apprwc(n: int, src, dst, w, v: int, diag: np.ndarray, method: str = "dense") -> np.ndarray:
    """Algorithm 1 (AppRWC), with the Laplacian solve taken exact.

    b = D^{1/2} (I - D^{1/2} 1 1^T D^{1/2} / vol) e_v;  z = LapSolve(L, b);
    y = (I - D^{1/2} 1 1^T D^{1/2} / vol) D^{1/2} z, an approximation of the v-th column of
    calL^+; then, from Theorem 3.1 (Eq. (3)),
    H_u = ((calL_v^{-1})_uu - (d_u/d_v) y_v + 2 sqrt(d_u/d_v) y_u) / pi_u for u != v and
    H_v = y_v / pi_v.  ``diag`` holds (calL_v^{-1})_uu (any value at index v is ignored).
    """
    if method == "dense":
        A = adjacency(n, src, dst, w)
        d = A.sum(axis=1)
    else:
        _, d = _sparse_laplacian(n, src, dst, w)
    vol = d.sum()
    sd = np.sqrt(d)

    def proj(x):
        return x - sd * (sd @ x) / vol

    ev = np.zeros(n)
    ev[v] = 1.0
    b = sd * proj(ev)
    z = lap_solve(n, src, dst, w, b, method, v)
    y = proj(sd * z)
    pi = d / vol
    H = (np.asarray(diag, dtype=np.float64) - (d / d[v]) * y[v] + 2.0 * np.sqrt(d / d[v]) * y) / pi
    H[v] = y[v] / pi[v]
    return H


def fastwalk_estimate(n: int, src, dst, w, v: int, counts: np.ndarray, l: int,
                      method: str = "dense") -> np.ndarray:
    """The last line of Algorithm 3: the visit totals of l sampled trees divided by l give
    the estimate of diag(calL_v^{-1}), which AppRWC turns into RWC."""
    t = np.asarray(counts, dtype=np.float64) / float(l)
    return apprwc(n, src, dst, w, v, t, method)


# ---------------------------------------------------------------------------------------
# Accuracy measures (Section 6.1)
# ---------------------------------------------------------------------------------------
def mean_relative_error(exact: np.ndarray, approx: np.ndarray) -> float:
    """MRE = (1/n) sum_u |H_u - H~_u| / H_u (Section 6.3)."""
    return float(np.mean(np.abs(exact - approx) / exact))


def kendall_tau_a(x: np.ndarray, y: np.ndarray) -> float:
    """2 (concordant - discordant) / (n (n - 1)), the rank measure of Section 6.1
    (computed by brute force over all pairs; for small n)."""
    x = np.asarray(x)
    y = np.asarray(y)
    n = x.shape[0]
    sx = np.sign(x[:, None] - x[None, :])
    sy = np.sign(y[:, None] - y[None, :])
    s = np.sum(np.triu(sx * sy, k=1))
    return float(2.0 * s / (n * (n - 1)))


# ---------------------------------------------------------------------------------------
# Groups of nodes (the generalisation named in the paper's Conclusion): random walk
# centrality of a set S, H_S = sum_i pi_i H_{i,S}, where H_{i,S} is the expected time for a
# walk from i to first reach S.
# ---------------------------------------------------------------------------------------
def hitting_times_to_set(n: int, src, dst, w, S) -> np.ndarray:
    """h_i = H_{i,S}: the first-step equations h_i = 1 + sum_k P_ik h_k for i outside S,
    h_i = 0 on S (Section 2.3's definition with S absorbing), by a dense solve."""
    A = adjacency(n, src, dst, w)
    P = A / A.sum(axis=1)[:, None]
    S = np.atleast_1d(np.asarray(S, dtype=np.int64))
    keep = np.setdiff1d(np.arange(n), S)
    h = np.zeros(n)
    h[keep] = np.linalg.solve(np.eye(keep.size) - P[np.ix_(keep, keep)], np.ones(keep.size))
    return h


def group_rwc(n: int, src, dst, w, S) -> float:
    """H_S = sum_i pi_i H_{i,S} with pi = d / vol."""
    d = adjacency(n, src, dst, w).sum(axis=1)
    return float((d / d.sum()) @ hitting_times_to_set(n, src, dst, w, S))


def grounded_inverse_diag_set(n: int, src, dst, w, S) -> np.ndarray:
    """d_u (L_S^{-1})_uu for u outside S (0 on S): the expected departures from u in one
    Wilson forest rooted at S, the root-set form of Lemma 5.2."""
    L = laplacian(adjacency(n, src, dst, w))
    d = np.diag(L).copy()
    S = np.atleast_1d(np.asarray(S, dtype=np.int64))
    keep = np.setdiff1d(np.arange(n), S)
    out = np.zeros(n)
    out[keep] = d[keep] * np.diag(np.linalg.inv(L[np.ix_(keep, keep)]))
    return out


def group_marginal_estimate(n: int, src, dst, w, S, t: np.ndarray) -> np.ndarray:
    """H_{S + u} for every u from H_S, the hitting times h to S and t_u, an estimate of
    d_u (L_S^{-1})_uu (the forests' visit totals over l): removing u from the system grounded
    at S is a rank-one update of its inverse, which gives
    H_{S + u} = H_S - d_u h_u^2 / (vol t_u) for u outside S, and H_S for u in S."""
    d = adjacency(n, src, dst, w).sum(axis=1)
    vol = d.sum()
    h = hitting_times_to_set(n, src, dst, w, S)
    hs = float((d / vol) @ h)
    S = np.atleast_1d(np.asarray(S, dtype=np.int64))
    out = np.full(n, hs)
    keep = np.setdiff1d(np.arange(n), S)
    t = np.asarray(t, dtype=np.float64)
    out[keep] = hs - d[keep] * h[keep] ** 2 / (vol * t[keep])
    return out
