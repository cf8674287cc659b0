"""CPU oracle for random walk centrality (RWC) and its FastWalk estimator.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the bench's
CPU-baseline leg may import or execute anything in this package.  The HIP library never
calls it and shares no code with it: the oracle has its own CSR construction, its own
Philox4x32-10, its own neighbour selection, its own counting and its own linear algebra.

Contents (each function cites the passage of the paper it follows):

* ``exact``     -- exact FP64 RWC from three independent characterisations (the hitting-time
                   definition of Section 2.3, Eq. (2) on the normalised Laplacian, and the
                   Laplacian pseudo-inverse formula of Section 2.2), the AppRWC assembly of
                   Algorithm 1 with an exact solve, and the quantities of Lemmas 5.1/5.2.
* ``wilson``    -- the serial FastWalk sampler of Algorithm 3 in plain C (``wilson.c``), with a
                   ctypes wrapper and the oracle's own CSR/CDF construction.
* ``gradient``  -- the exact gradient of sum_j g_j RWC_j with respect to the edge weights,
                   its JL-sketch estimator, and a float64 autograd cross-check.

Nothing here is tuned for speed.
"""
