"""Seeded synthetic undirected graphs shaped like the paper's workloads.

The paper evaluates on large SNAP social networks (its Table 1: power-law degree
distributions, average degree 5 to 76, millions of nodes).  Those datasets are not
available here, so these generators stand in for them:

* Erdos-Renyi G(n, p) restricted to its largest connected component,
* Barabasi-Albert preferential attachment (Batagelj and Brandes, "Efficient generation
  of large random networks", Phys. Rev. E 71, 2005, the edge-list copying model),
* 2D grid meshes with a fraction of the edges deleted uniformly at random (road-like),
* R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) with a seeded random relabelling.

Every generator returns a simple graph: no self-loops, no duplicate edges, and, after
``largest_component``, connected with nodes relabelled 0..n-1 in increasing original id
(the paper evaluates on the largest connected component only, Section 6.1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


@dataclasses.dataclass
class EdgeList:
    n: int
    src: np.ndarray          # int32 [m]
    dst: np.ndarray          # int32 [m]
    w: np.ndarray | None     # float32 [m] or None for unit weights
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def with_weights(self, w: np.ndarray | None, name: str | None = None) -> "EdgeList":
        return EdgeList(self.n, self.src, self.dst, w, name or self.name)


def _simple(n: int, a: np.ndarray, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Drop self-loops and duplicate undirected edges; return (lo, hi) pairs sorted."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = np.unique(lo * n + hi)
    return (key // n).astype(np.int64), (key % n).astype(np.int64)


def largest_component(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray | None = None,
                      name: str = "") -> EdgeList:
    """Restrict to the largest connected component, relabelled in increasing original id."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if n == 0:
        return EdgeList(0, src.astype(np.int32), dst.astype(np.int32), w, name)
    adj = sp.coo_matrix((np.ones(src.shape[0], dtype=np.int8), (src, dst)), shape=(n, n))
    ncomp, label = csg.connected_components(adj, directed=False)
    if ncomp == 1:
        keep_nodes = np.ones(n, dtype=bool)
    else:
        sizes = np.bincount(label, minlength=ncomp)
        big = int(np.argmax(sizes))
        keep_nodes = label == big
    new_id = np.cumsum(keep_nodes) - 1
    keep_edges = keep_nodes[src] & keep_nodes[dst]
    s2 = new_id[src[keep_edges]].astype(np.int32)
    d2 = new_id[dst[keep_edges]].astype(np.int32)
    w2 = None if w is None else np.asarray(w, dtype=np.float32)[keep_edges]
    return EdgeList(int(keep_nodes.sum()), s2, d2, w2, name)


def uniform_weights(m: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Edge weights drawn i.i.d. from U[lo, hi], stored as float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=m).astype(np.float32)


def erdos_renyi_lcc(n: int, avg_deg: float, seed: int) -> EdgeList:
    """G(n, p) with p = avg_deg / (n - 1), largest connected component."""
    rng = np.random.default_rng(seed)
    p = avg_deg / (n - 1)
    if n <= 20000:
        iu, ju = np.triu_indices(n, k=1)
        keep = rng.random(iu.shape[0]) < p
        a, b = iu[keep], ju[keep]
    else:
        # Number of edges is Binomial(n(n-1)/2, p); endpoints drawn uniformly, then
        # duplicates removed (a negligible deviation from G(n, p) at this density).
        total = n * (n - 1) // 2
        m = rng.binomial(total, p)
        a = rng.integers(0, n, size=int(m * 1.02) + 16)
        b = rng.integers(0, n, size=a.shape[0])
    lo, hi = _simple(n, a, b)
    return largest_component(n, lo, hi, None, f"er{n}_d{avg_deg:g}_s{seed}")


def barabasi_albert(n: int, m: int, seed: int) -> EdgeList:
    """Preferential attachment by edge-list copying (Batagelj-Brandes).

    Slot 2k holds the new node k // m; slot 2k + 1 copies a uniformly chosen earlier slot
    r in [0, 2k] (inclusive), which picks an existing node with probability proportional
    to its current degree.  Self-loops and repeated edges are dropped and the largest
    component kept.
    """
    rng = np.random.default_rng(seed)
    nm = n * m
    k = np.arange(nm, dtype=np.int64)
    r = rng.integers(0, 2 * k + 1)            # r_k uniform in [0, 2k]
    ptr = np.empty(2 * nm, dtype=np.int64)
    ptr[0::2] = np.arange(0, 2 * nm, 2)       # even slots are fixed points
    ptr[1::2] = r
    # Resolve the copy chains by pointer jumping: every odd slot points strictly left.
    while True:
        nxt = ptr[ptr]
        if np.array_equal(nxt, ptr):
            break
        ptr = nxt
    val = ptr // 2 // m                       # even slot 2k holds node k // m
    a = val[0::2]
    b = val[1::2]
    lo, hi = _simple(n, a, b)
    return largest_component(n, lo, hi, None, f"ba{n}_m{m}_s{seed}")


def grid_with_deletions(n: int, frac: float, seed: int) -> EdgeList:
    """r x c grid with r = floor(sqrt(n)), c = ceil(n / r); a fraction `frac` of the edges
    is deleted uniformly at random; largest component kept."""
    rng = np.random.default_rng(seed)
    r = max(1, int(math.isqrt(n)))
    c = max(1, -(-n // r))
    ids = np.arange(r * c, dtype=np.int64).reshape(r, c)
    ha = ids[:, :-1].ravel()
    hb = ids[:, 1:].ravel()
    va = ids[:-1, :].ravel()
    vb = ids[1:, :].ravel()
    a = np.concatenate([ha, va])
    b = np.concatenate([hb, vb])
    ndel = int(round(frac * a.shape[0]))
    keep = np.ones(a.shape[0], dtype=bool)
    if ndel:
        keep[rng.choice(a.shape[0], size=ndel, replace=False)] = False
    lo, hi = _simple(r * c, a[keep], b[keep])
    return largest_component(r * c, lo, hi, None, f"grid{r}x{c}_del{frac:g}_s{seed}")


def rmat_lcc(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> EdgeList:
    """R-MAT with 2**scale nodes and edge_factor * 2**scale edge draws; seeded random
    relabelling, duplicate and self-loop removal, largest component."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    ne = edge_factor * n
    row = np.zeros(ne, dtype=np.int64)
    col = np.zeros(ne, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    chunk = 1 << 22
    for lo_i in range(0, ne, chunk):
        hi_i = min(ne, lo_i + chunk)
        rr = np.zeros(hi_i - lo_i, dtype=np.int64)
        cc = np.zeros(hi_i - lo_i, dtype=np.int64)
        for bit in range(scale):
            u = rng.random(hi_i - lo_i)
            rbit = u >= ab                                   # quadrants c, d
            cbit = ((u >= a) & (u < ab)) | (u >= abc)        # quadrants b, d
            rr |= rbit.astype(np.int64) << bit
            cc |= cbit.astype(np.int64) << bit
        row[lo_i:hi_i] = rr
        col[lo_i:hi_i] = cc
    perm = rng.permutation(n)
    row = perm[row]
    col = perm[col]
    lo, hi = _simple(n, row, col)
    del row, col
    return largest_component(n, lo, hi, None, f"rmat{scale}_ef{edge_factor}_s{seed}")


def complete_graph(n: int) -> EdgeList:
    a, b = np.triu_indices(n, k=1)
    return EdgeList(n, a.astype(np.int32), b.astype(np.int32), None, f"K{n}")


def star_graph(n: int) -> EdgeList:
    """Centre 0 joined to leaves 1..n-1."""
    leaves = np.arange(1, n, dtype=np.int32)
    return EdgeList(n, np.zeros(n - 1, dtype=np.int32), leaves, None, f"star{n}")


def cycle_graph(n: int) -> EdgeList:
    a = np.arange(n, dtype=np.int32)
    return EdgeList(n, a, ((a + 1) % n).astype(np.int32), None, f"C{n}")


def path_graph(n: int) -> EdgeList:
    a = np.arange(n - 1, dtype=np.int32)
    return EdgeList(n, a, a + 1, None, f"P{n}")


def disjoint_union(parts: list[EdgeList], isolated: int = 0) -> EdgeList:
    """The parts side by side (part k's ids shifted by the sizes of parts 0..k-1), then
    `isolated` nodes without edges: a graph of len(parts) + isolated connected components
    (each part connected).  Weights are kept when every part has them, else unit weights."""
    src, dst, ws, off = [], [], [], 0
    for g in parts:
        src.append(g.src.astype(np.int64) + off)
        dst.append(g.dst.astype(np.int64) + off)
        ws.append(g.w)
        off += g.n
    w = np.concatenate(ws).astype(np.float32) if all(x is not None for x in ws) else None
    return EdgeList(off + isolated, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32), w,
                    "+".join(g.name for g in parts) + (f"+{isolated} isolated" if isolated else ""))


def batch_mix(count: int, n_lo: float, n_hi: float, seed: int, w_lo: float = 0.5,
              w_hi: float = 2.0) -> list[EdgeList]:
    """`count` graphs of uneven size: n log-uniform in [n_lo, n_hi]; the first half
    Barabasi-Albert with 3 edges per new node, the second half grids with 10% of the
    edges deleted; weights U[w_lo, w_hi] in float32."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    out = []
    for i, ng in enumerate(sizes):
        gseed = int(seed * 1000003 + i)
        if i < count // 2:
            g = barabasi_albert(int(ng), 3, gseed)
        else:
            g = grid_with_deletions(int(ng), 0.1, gseed)
        w = uniform_weights(g.m, w_lo, w_hi, gseed + 17)
        out.append(g.with_weights(w, g.name))
    return out
