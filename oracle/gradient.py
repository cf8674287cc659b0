"""Gradient of l(w) = sum_j g_j RWC_j with respect to the edge weights (CPU oracle, test-only).

RWC is written as H_j = vol L^+_jj - 2 (L^+ d)_j + d^T L^+ d / vol (Eq. (2) combined with the
pseudo-inverse identity of Section 3).  Differentiating with dL/dw_e = b_e b_e^T (b_e from the
incidence matrix of Section 2.2), dL^+/dw_e = -L^+ b_e b_e^T L^+ (the graph stays connected),
dd/dw_e = e_a + e_b and dvol/dw_e = 2 gives, with A = L^+ g, B = L^+ d, G = sum g,
trGL = sum_j g_j L^+_jj, dLd = d^T B, Q_e = sum_j g_j (L^+ b_e)_j^2 and, for an edge e = (a, b),
D_X = X_a - X_b, S_X = X_a + X_b:

    dl/dw_e = 2 trGL - vol Q_e + 2 D_A D_B - 2 S_A + G ((2 S_B - D_B^2) / vol - 2 dLd / vol^2).

The paper does not differentiate RWC; this is the adjoint of its quantity.  The sketched
variant replaces Q_e and trGL by Johnson-Lindenstrauss / Hutchinson estimates built from the
same k Rademacher probes r_i restricted to the support of g (g >= 0):
Z = L^+ G^{1/2} R^T, Q^_e = (1/k) sum_i (b_e^T Z_i)^2, trGL^ = (1/k) sum_i (G^{1/2} r_i)^T Z_i.
"""
from __future__ import annotations

import numpy as np

from .exact import adjacency, laplacian, laplacian_pinv


def _edge_terms(n, src, dst, w, g):
    A_ = adjacency(n, src, dst, w)
    d = A_.sum(axis=1)
    vol = d.sum()
    Lp = laplacian_pinv(laplacian(A_))
    g = np.asarray(g, dtype=np.float64)
    A = Lp @ g
    B = Lp @ d
    a = np.asarray(src, dtype=np.int64)
    b = np.asarray(dst, dtype=np.int64)
    return d, vol, Lp, g, A, B, a, b


def _assemble(vol, g, A, B, a, b, Q, trGL, dLd):
    G = g.sum()
    DA = A[a] - A[b]
    DB = B[a] - B[b]
    SA = A[a] + A[b]
    SB = B[a] + B[b]
    return (2.0 * trGL - vol * Q + 2.0 * DA * DB - 2.0 * SA
            + G * ((2.0 * SB - DB * DB) / vol - 2.0 * dLd / (vol * vol)))


def grad_exact(n: int, src, dst, w, g) -> np.ndarray:
    """dl/dw_e for every input edge, dense FP64, in input-edge order."""
    d, vol, Lp, g, A, B, a, b = _edge_terms(n, src, dst, w, g)
    Y = Lp[:, a] - Lp[:, b]                       # column e is L^+ b_e
    Q = (g[:, None] * Y * Y).sum(axis=0)
    trGL = float(g @ np.diag(Lp))
    return _assemble(vol, g, A, B, a, b, Q, trGL, float(d @ B))


def grad_sketch(n: int, src, dst, w, g, R: np.ndarray) -> np.ndarray:
    """Sketched gradient from the k x n probe matrix R (rows r_i; entries are used only on
    the support of g).  Requires g >= 0."""
    d, vol, Lp, g, A, B, a, b = _edge_terms(n, src, dst, w, g)
    if np.any(g < 0):
        raise ValueError("the sketch needs g >= 0")
    k = R.shape[0]
    Y = np.sqrt(g)[None, :] * R                   # rows G^{1/2} r_i
    Z = Lp @ Y.T                                  # n x k
    Dz = Z[a, :] - Z[b, :]
    Q = (Dz * Dz).sum(axis=1) / k
    trGL = float(np.sum(Y.T * Z) / k)
    return _assemble(vol, g, A, B, a, b, Q, trGL, float(d @ B))


def loss(n: int, src, dst, w, g) -> float:
    """l(w) = sum_j g_j RWC_j from the dense pseudo-inverse form."""
    A_ = adjacency(n, src, dst, w)
    d = A_.sum(axis=1)
    vol = d.sum()
    Lp = laplacian_pinv(laplacian(A_))
    Ld = Lp @ d
    H = vol * np.diag(Lp) - 2.0 * Ld + (d @ Ld) / vol
    return float(np.asarray(g, dtype=np.float64) @ H)


def grad_autograd(n: int, src, dst, w, g) -> np.ndarray:
    """The same gradient by reverse-mode automatic differentiation (torch, float64, CPU) of
    the normalised-Laplacian form of Eq. (2): H_u = (calL^+)_uu / pi_u, with calL^+ obtained
    from a dense inverse of calL + s s^T / vol (s = D^{1/2} 1) minus that rank-one term."""
    import torch

    src_t = torch.as_tensor(np.asarray(src, dtype=np.int64))
    dst_t = torch.as_tensor(np.asarray(dst, dtype=np.int64))
    wt = torch.tensor(np.ones(len(src)) if w is None else np.asarray(w, dtype=np.float64),
                      dtype=torch.float64, requires_grad=True)
    A = torch.zeros(n, n, dtype=torch.float64)
    A = A.index_put((src_t, dst_t), wt, accumulate=True)
    A = A.index_put((dst_t, src_t), wt, accumulate=True)
    d = A.sum(dim=1)
    vol = d.sum()
    s = torch.sqrt(d)
    Ln = torch.eye(n, dtype=torch.float64) - A / (s[:, None] * s[None, :])
    P = torch.outer(s, s) / vol                    # projector on the null space of calL
    Lnp = torch.linalg.inv(Ln + P) - P
    H = torch.diagonal(Lnp) / (d / vol)
    lval = (torch.as_tensor(np.asarray(g, dtype=np.float64)) * H).sum()
    lval.backward()
    return wt.grad.detach().numpy().copy()
