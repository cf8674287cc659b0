"""Writes ba20k_exact_rwc.txt: exact FP64 random walk centrality of BA(n = 20 000, m = 5, seed
1002, unit weights) at 2000 seeded sample nodes plus the pivot, from the CPU oracle's
closed form H_u = vol L^+_uu - 2 (L^+ d)_u + d^T L^+ d / vol (Section 2.2 pseudo-inverse,
Section 3 identity).  Run from the repository root: python tests/golden/make_ba20k_exact.py
(about a minute on 8 cores; the dense factor takes 3.2 GB)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rwcgen as G  # noqa: E402
from oracle import exact as E  # noqa: E402

N, M_EDGES, GRAPH_SEED, PICK_SEED, PICKS = 20_000, 5, 1002, 7, 2000


def main():
    g = G.barabasi_albert(N, M_EDGES, GRAPH_SEED)
    h = E.rwc_laplacian_pinv_cholesky(g.n, g.src, g.dst, g.w)
    v = E.pivot_of(g.n, g.src, g.dst, g.w)
    nodes = np.unique(np.concatenate([[v], np.random.default_rng(PICK_SEED).choice(g.n, PICKS, replace=False)]))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ba20k_exact_rwc.txt")
    with open(out, "w") as f:
        f.write(f"# exact RWC of BA(n={N}, m={M_EDGES}, seed={GRAPH_SEED}), unit weights; pivot {v}\n")
        f.write("# written by tests/golden/make_ba20k_exact.py (oracle.exact.rwc_laplacian_pinv_cholesky)\n")
        f.write("# node | RWC\n")
        for u in nodes:
            f.write(f"{int(u)} | {float(h[u])!r}\n")


if __name__ == "__main__":
    main()
