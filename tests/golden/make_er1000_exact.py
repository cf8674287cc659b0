"""Writes er1000_exact_rwc.txt: exact FP64 random walk centrality of every node of the largest
component of ER(n = 1000, average degree 8, seed 1001), unit weights, from the CPU oracle's
closed form H_u = vol L^+_uu - 2 (L^+ d)_u + d^T L^+ d / vol (Section 2.2 pseudo-inverse,
Section 3 identity).  Run from the repository root: python tests/golden/make_er1000_exact.py"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rwcgen as G  # noqa: E402
from oracle import exact as E  # noqa: E402


def main():
    g = G.erdos_renyi_lcc(1000, 8, 1001)
    h = E.rwc_laplacian_pinv(g.n, g.src, g.dst, g.w)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "er1000_exact_rwc.txt")
    with open(out, "w") as f:
        f.write(f"# exact RWC of the ER(n=1000, d=8, seed=1001) largest component ({g.n} nodes), unit weights\n")
        f.write("# written by tests/golden/make_er1000_exact.py (oracle.exact.rwc_laplacian_pinv)\n")
        f.write("# node | RWC\n")
        for u in range(g.n):
            f.write(f"{u} | {float(h[u])!r}\n")


if __name__ == "__main__":
    main()
