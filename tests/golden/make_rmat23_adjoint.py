"""Writes rmat23_adjoint_grad.txt: the gradient of l(w) = sum over 1000 targets of RWC_j with
respect to the edge weights of the R-MAT scale-23 workload (largest component of R-MAT(scale 23,
5 draws per node, (a, b, c) = (.57, .19, .19), seed 1005), weights U[1, 4] seed 1006), at 24
sampled input edges, from the CPU oracle only: oracle.gradient.grad_at_edges_sparse with the
64 Rademacher probe columns of oracle.gradient.probe_columns (k = 64, probe seed 2006), every
L^+ y a grounded sparse CG solve to relative residual 1e-11.  Targets: 1000 distinct nodes drawn
by numpy's default_rng(7), g = 1 on each.  Edges: 24 distinct input edges drawn by
default_rng(8).

Run from the repository root: python tests/golden/make_rmat23_adjoint.py [workers]
(about 15 minutes on 8 cores with 6 workers; 10-15 GB of memory)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rwcgen as G  # noqa: E402
from oracle import gradient as GR  # noqa: E402

SCALE, EDGE_FACTOR, ABC, GRAPH_SEED, WEIGHT_SEED = 23, 5, (0.57, 0.19, 0.19), 1005, 1006
TARGETS, TARGET_SEED, K, PROBE_SEED, EDGES, EDGE_SEED, RTOL = 1000, 7, 64, 2006, 24, 8, 1e-11


def main(workers: int = 6):
    t0 = time.time()
    g = G.rmat_lcc(SCALE, EDGE_FACTOR, *ABC, GRAPH_SEED)
    g = g.with_weights(G.uniform_weights(g.m, 1.0, 4.0, WEIGHT_SEED))
    print(f"graph n={g.n} m={g.m} ({time.time() - t0:.0f} s)", flush=True)
    targets = np.random.default_rng(TARGET_SEED).choice(g.n, size=TARGETS, replace=False).astype(np.int32)
    gv = np.ones(TARGETS)
    edges = np.random.default_rng(EDGE_SEED).choice(g.m, size=EDGES, replace=False)
    cols = GR.probe_columns(g.n, targets, gv, K, PROBE_SEED)
    print(f"{len(cols)} probe columns ({time.time() - t0:.0f} s)", flush=True)
    grad = GR.grad_at_edges_sparse(g.n, g.src, g.dst, g.w, targets, gv, edges, cols=cols, rtol=RTOL,
                                   workers=workers)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat23_adjoint_grad.txt")
    with open(out, "w") as f:
        f.write(f"# d(sum_j RWC_j)/dw_e on the R-MAT scale-{SCALE} largest component (n={g.n}, m={g.m}), "
                f"w ~ U[1, 4] seed {WEIGHT_SEED}\n")
        f.write(f"# {TARGETS} targets default_rng({TARGET_SEED}), g = 1; sketch k = {K}, probe seed {PROBE_SEED}; "
                f"CG rtol {RTOL}\n")
        f.write("# written by tests/golden/make_rmat23_adjoint.py (oracle.gradient.grad_at_edges_sparse)\n")
        f.write("# edge | src | dst | grad\n")
        for e, val in zip(edges, grad):
            f.write(f"{int(e)} | {int(g.src[e])} | {int(g.dst[e])} | {float(val)!r}\n")
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
