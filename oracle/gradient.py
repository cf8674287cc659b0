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


# ---------------------------------------------------------------------------------------
# Probe columns shared by the exact and sketched forms, and a sparse evaluation at sampled
# edges for graphs too large for dense matrices.
# ---------------------------------------------------------------------------------------
def probe_columns(n: int, targets, gvals, k: int, seed: int):
    """Columns (c_i, y_i) with Q_e ~ sum_i c_i (b_e^T L^+ y_i)^2 and trGL ~ sum_i c_i y_i^T L^+ y_i.

    k = 0: y = sqrt|g_j| e_j, c = sign(g_j) for every target (exact).
    k > 0: for each sign class of g present (positive first), k Rademacher probes
    y_i = sqrt(|g|) r_i restricted to that class, c_i = +-1/k.  The sign of probe i at node u is
    bit 0 of word 0 of Philox4x32-10 on the counter (i, u, 0, 2^32 - 1) with key `seed`;
    probes of the negative class are numbered k .. 2k - 1.
    """
    from .wilson import philox4x32_10
    targets = np.asarray(targets, dtype=np.int64)
    gvals = np.asarray(gvals, dtype=np.float64)
    cols = []
    if k == 0:
        for t, gv in zip(targets, gvals):
            y = np.zeros(n)
            y[t] = np.sqrt(abs(gv))
            cols.append((float(np.sign(gv)), y))
        return cols
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    for cls in (0, 1):
        sel = gvals > 0 if cls == 0 else gvals < 0
        if not np.any(sel):
            continue
        for i in range(k):
            probe = cls * k + i
            y = np.zeros(n)
            for t, gv in zip(targets[sel], gvals[sel]):
                o0 = philox4x32_10([probe, int(t), 0, 0xFFFFFFFF], key)[0]
                y[t] = (-1.0 if (o0 & 1) else 1.0) * np.sqrt(abs(gv))
            cols.append(((1.0 if cls == 0 else -1.0) / k, y))
    return cols


def grad_from_probes(n: int, src, dst, w, g, cols) -> np.ndarray:
    """Dense gradient with Q_e and trGL taken from the probe columns."""
    d, vol, Lp, g, A, B, a, b = _edge_terms(n, src, dst, w, g)
    Q = np.zeros(len(a))
    trGL = 0.0
    for c, y in cols:
        z = Lp @ y
        dz = z[a] - z[b]
        Q += c * dz * dz
        trGL += c * float(y @ z)
    return _assemble(vol, g, A, B, a, b, Q, trGL, float(d @ B))


_POOL_GRAPH = None


def _pool_init(n, src, dst, w, rtol):
    global _POOL_GRAPH
    _POOL_GRAPH = (n, src, dst, w, rtol)


def _pool_pinv(y):
    n, src, dst, w, rtol = _POOL_GRAPH
    from .exact import lap_solve
    yc = y - y.mean()
    z = lap_solve(n, src, dst, w, yc, "sparse_cg", rtol=rtol)
    return z - z.mean()


def grad_at_edges_sparse(n: int, src, dst, w, targets, gvals, edges, cols=None, rtol: float = 1e-14,
                         workers: int = 1) -> np.ndarray:
    """dl/dw_e for the input edges `edges` from sparse conjugate-gradient solves (SciPy), for
    graphs too large for dense matrices.  cols=None evaluates Q_e and trGL exactly (one solve
    per sampled edge and per target); otherwise from the given probe columns.  Each L^+ y is
    one grounded CG solve to relative residual `rtol`, centred; with workers > 1 the probe
    columns' solves run in that many processes (the same solves, in any order)."""
    from .exact import _sparse_laplacian, lap_solve
    L, d = _sparse_laplacian(n, src, dst, w)
    vol = d.sum()
    targets = np.asarray(targets, dtype=np.int64)
    gvals = np.asarray(gvals, dtype=np.float64)
    g = np.zeros(n)
    g[targets] = gvals

    def pinv(y):
        yc = y - y.mean()
        z = lap_solve(n, src, dst, w, yc, "sparse_cg", rtol=rtol)
        return z - z.mean()

    A = pinv(g)
    B = pinv(d)
    a = np.asarray(src, dtype=np.int64)[edges]
    b = np.asarray(dst, dtype=np.int64)[edges]
    if cols is None:
        trGL = 0.0
        for t, gv in zip(targets, gvals):
            e = np.zeros(n)
            e[t] = 1.0
            trGL += gv * pinv(e)[t]
        Q = np.zeros(len(edges))
        for i, (ai, bi) in enumerate(zip(a, b)):
            be = np.zeros(n)
            be[ai], be[bi] = 1.0, -1.0
            y = pinv(be)
            Q[i] = float(g @ (y * y))
    else:
        Q = np.zeros(len(edges))
        trGL = 0.0
        if workers > 1:
            import concurrent.futures as cf
            with cf.ProcessPoolExecutor(max_workers=workers, initializer=_pool_init,
                                        initargs=(n, src, dst, w, rtol)) as ex:
                zs = list(ex.map(_pool_pinv, [y for _, y in cols]))
        else:
            zs = [pinv(y) for _, y in cols]
        for (c, y), z in zip(cols, zs):
            dz = z[a] - z[b]
            Q += c * dz * dz
            trGL += c * float(y @ z)
    return _assemble(vol, g, A, B, a, b, Q, trGL, float(d @ B))
