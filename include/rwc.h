/*
 * rwc.h -- C ABI of the MI355X FastWalk library: random walk centrality (RWC) from rooted
 * spanning trees sampled with Wilson's algorithm (Liu, Xie, Zehmakan, Zhang, "Efficient
 * Algorithms for Computing Random Walk Centrality", Section 5, Algorithm 3), assembled by
 * the pivot reformulation of Theorem 3.1 / Algorithm 1 (AppRWC).
 *
 * Conventions shared by every entry point
 *  - Every pointer argument named *_dev, and every pointer inside rwc_csr /
 *    rwc_sample_outputs unless stated otherwise, is a DEVICE pointer owned by the caller.
 *    The library never allocates device memory: each call that needs scratch space takes a
 *    caller-owned workspace whose size is returned by the matching *_workspace query.
 *    Workspaces must be 256-byte aligned.
 *  - `stream` is a hipStream_t passed as void*; all device work is ordered on it.
 *  - Return value: RWC_OK (0) or a negative rwc_status.  On an argument error no output is
 *    touched.  No exception or abort crosses the ABI.  rwc_last_error() gives a
 *    human-readable detail of the most recent failure on the calling thread.
 *  - Graph semantics: undirected, no self-loops, no repeated edges, connected (the paper
 *    works on the largest connected component of each graph, Section 6.1).  Edge weights,
 *    when given, are float32 values in [0.5, 65536); the walk moves from u to a neighbour
 *    with probability w_uv / d_u where d_u is the weighted degree (the paper's unweighted
 *    walk of Section 2.3 is the case w = 1).
 */
#ifndef RWC_H
#define RWC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rwc_status {
    RWC_OK = 0,
    RWC_ERR_INVALID_ARG = -1,      /* null pointer, negative size, bad flag combination      */
    RWC_ERR_NODE_RANGE = -2,       /* an edge endpoint or root id outside [0, n)             */
    RWC_ERR_SELF_LOOP = -3,        /* an edge (u, u)                                         */
    RWC_ERR_DUP_EDGE = -4,         /* the same undirected edge listed twice                  */
    RWC_ERR_WEIGHT_RANGE = -5,     /* a weight outside [0.5, 65536) or not finite, a weighted
                                      degree of 2^29 or more, or total weight of 2^40 or more */
    RWC_ERR_DISCONNECTED = -6,     /* more than one connected component (or an isolated node)*/
    RWC_ERR_TOO_LARGE = -7,        /* n >= 2^31 - 1, 2m >= 2^31, or an index space overflow  */
    RWC_ERR_WORKSPACE = -8,        /* workspace null, misaligned or smaller than required    */
    RWC_ERR_STEP_LIMIT = -9,       /* a tree needed more walk steps than max_steps_per_tree  */
    RWC_ERR_COUNT_OVERFLOW = -10,  /* a node departed 2^24 times within one tree             */
    RWC_ERR_NOT_CONVERGED = -11,   /* the pivot/adjoint solve missed its tolerance           */
    RWC_ERR_HIP = -12,             /* a HIP runtime call failed                              */
    RWC_ERR_BREAKDOWN = -13        /* FastChol: a non-positive pivot in the incomplete factor */
} rwc_status;

/* A graph in device memory, produced by rwc_build_csr.  All pointers point into the
 * workspace given to rwc_build_csr, which must outlive every use of the struct. */
typedef struct rwc_csr {
    int32_t n;             /* nodes                                                         */
    int32_t pivot;         /* node of largest weighted degree, ties to the smallest id (an
                              input id; its internal index is pivot_index)                  */
    int64_t m;             /* undirected edges (= input edges)                              */
    int64_t nnz;           /* 2m directed CSR entries                                       */
    int32_t weighted;      /* 1 if the graph was built with weights                         */
    int32_t max_degree;    /* largest number of neighbours                                  */
    double vol;            /* sum of weighted degrees (2m for unit weights)                 */
    uint64_t vol_fixed;    /* vol * 2^24, exact                                             */
    /* The arrays below are in the graph's internal order (see node_id): row x, strength[x],
       rec[16 x ..] and the ids in col and bfs_order are internal indices.  Every per-node
       array a caller passes to or gets from the library is indexed by input id.           */
    int32_t* row_ptr;      /* [n + 1] CSR offsets                                           */
    int32_t* col;          /* [nnz] internal indices of the neighbours, ordered within each
                              row by ascending input id                                     */
    float* weight;         /* [nnz] weight of each entry (1 for unweighted graphs)          */
    int32_t* edge_id;      /* [nnz] index of the input edge each entry came from            */
    uint64_t* cdf;         /* [nnz] inclusive prefix sums within each row of the integer
                              weights W_e = w_e * 2^24 (NULL for unweighted graphs)         */
    double* strength;      /* [n] weighted degree d_u                                       */
    uint32_t* rec;         /* [16 n] 64-byte node records: word 0 the degree, word 1 the row
                              offset, word 2 the node's input id; unweighted rows: the first
                              13 neighbours in words 3..15; weighted rows: the first 3 in
                              words 3..5, the row's total (last CDF value) in words 6..7 and
                              the first 3 CDF values in words 8..13; unused words are zero  */
    int32_t* bfs_order;    /* [n] nodes in breadth-first order from the pivot: the order in
                              which walker teams take start nodes                          */
    int32_t bfs_depth;     /* largest hop distance from the pivot (its eccentricity in its
                              component)                                                    */
    int32_t components;    /* connected components (1 unless built with
                              RWC_BUILD_ALLOW_DISCONNECTED)                                 */
    int32_t* node_id;      /* [n] input id of internal index x                              */
    int32_t* node_index;   /* [n] internal index of input id u                              */
    int32_t pivot_index;   /* internal index of the pivot                                   */
    int32_t internal_order;/* 1: nodes stored by descending weighted degree, ties by input
                              id (graphs whose largest degree exceeds four times the mean);
                              0: internal index = input id.  Placement only: no result
                              depends on it                                                 */
    int32_t* component;    /* [n] by input id: the smallest input id of the node's
                              connected component                                           */
} rwc_csr;

/* Bytes of workspace rwc_build_csr needs for n nodes and m edges (weighted != 0 if w will
 * be given).  The first rwc_csr_persistent_bytes() of it hold the CSR and must be kept; the
 * rest is scratch that is free again when rwc_build_csr returns. */
int rwc_build_csr_workspace(int32_t n, int64_t m, int32_t weighted, size_t* bytes);
int rwc_csr_persistent_bytes(int32_t n, int64_t m, int32_t weighted, size_t* bytes);

/* Builds the symmetric CSR used by every other call: rows sorted by neighbour id, weighted
 * degrees d, vol, the integer CDF rows that RandomNeighbor (Algorithm 3) samples from, and
 * the pivot of Section 6.1 (largest degree).  Validates the input and checks connectivity.
 *   src_dev, dst_dev  int32 [m] edge endpoints (device)
 *   w_dev             float32 [m] weights (device) or NULL for unit weights
 * Synchronises `stream` before returning (it reads back a status word and the scalars). */
int rwc_build_csr(int32_t n, int64_t m, const int32_t* src_dev, const int32_t* dst_dev,
                  const float* w_dev, void* ws, size_t ws_bytes, rwc_csr* out, void* stream);

/* Build flags. */
#define RWC_BUILD_ALLOW_DISCONNECTED 1u  /* accept several connected components (isolated nodes
                                            included) for forests rooted at a set that meets
                                            every component (Conclusion: groups of nodes; one
                                            root per component makes every walk end): the CSR
                                            records `components` and `component`, bfs_order
                                            lists the pivot's component first, then the other
                                            nodes in internal order.  Calls that need a
                                            connected graph (a single root: the pivot estimate,
                                            trap walks, FastChol, the adjoint, the autotuners
                                            and unrooted sampling) return RWC_ERR_DISCONNECTED
                                            for such a CSR; a root set that misses a component
                                            is reported by the device as RWC_ERR_DISCONNECTED */

/* rwc_build_csr with flags (0 or RWC_BUILD_ALLOW_DISCONNECTED; other bits are
 * RWC_ERR_INVALID_ARG).  rwc_build_csr(...) is rwc_build_csr_ex(..., 0, ...). */
int rwc_build_csr_ex(int32_t n, int64_t m, const int32_t* src_dev, const int32_t* dst_dev,
                     const float* w_dev, uint32_t flags, void* ws, size_t ws_bytes, rwc_csr* out,
                     void* stream);

/* Sampling flags. */
#define RWC_SAMPLE_ACCUMULATE    1u  /* add to counts / counts_sq / total_steps instead of
                                        overwriting them                                    */
#define RWC_SAMPLE_PERSISTENT    2u  /* batched: one persistent launch whose waves pop (graph,
                                        tree block) work items from a device queue          */
#define RWC_SAMPLE_GRAPH_CAPTURE 4u  /* run the call's launches as a hipGraph: captured and
                                        instantiated on the first call with a given set of
                                        graphs, parameters, workspace and outputs, and replayed
                                        (after a fresh upload of the call's argument tables) by
                                        later calls with the same set.  The library keeps at
                                        most 8 such graphs (least recently used dropped);
                                        rwc_release_cached_graphs frees them                 */
#define RWC_SAMPLE_BFS_STARTS    8u  /* walker teams take start nodes in breadth-first order
                                        from the root instead of ascending ids (same forest) */
#define RWC_SAMPLE_ID_STARTS   256u  /* walker teams take start nodes by ascending id.  With
                                        neither this nor BFS, graphs with spread starts take
                                        them breadth-first when the call has several graphs
                                        and queues at least twice the waves the device
                                        holds, ascending otherwise (same forest)            */
#define RWC_SAMPLE_SPREAD_STARTS 16u /* each walker of a team takes start nodes from its own
                                        contiguous range of the start order (same forest)   */
#define RWC_SAMPLE_SHARED_STARTS 32u /* a team's walkers take consecutive start positions.
                                        With neither this nor SPREAD, each graph gets spread
                                        starts if its bfs_depth exceeds 32 (long walks, e.g.
                                        meshes), shared starts otherwise                    */
#define RWC_SAMPLE_PATH_RING     64u /* team kernel keeps each walker's newest path nodes and
                                        their departure counts in LDS, so loop erasure and
                                        attachment of them are single stores with no read
                                        (same forest)                                       */
#define RWC_SAMPLE_NO_PATH_RING 128u /* team kernel without that ring.  With neither, the
                                        ring is used unless the call's waves fill two thirds
                                        of the device or more, some graph is weighted with
                                        more than 16 entries per node, and no graph has
                                        spread starts (same forest)                         */

#define RWC_SAMPLE_NO_LDS_STATE 512u /* keep every graph's tree state in HBM.  Without it,
                                        a call whose graphs all use walker teams and all fit
                                        (64 / W trees of n 8-byte words in 48 KB of LDS; at
                                        most 2^24 samples) grows its trees in LDS instead:
                                        no HBM tree slots, LDS accesses for every state read
                                        and write (same forest)                            */

typedef struct rwc_sample_params {
    uint64_t seed;               /* Philox key (seed mod 2^32, seed >> 32)                 */
    int64_t sample_begin;        /* global index of the first sample                      */
    int64_t num_samples;         /* trees per graph (l in Algorithm 3)                    */
    int32_t root;                /* -1: each graph's pivot; otherwise the root (1 graph)   */
    uint32_t flags;              /* RWC_SAMPLE_*                                          */
    int32_t trees_in_flight;     /* trees resident at once per graph; 0 = automatic: all
                                    trees, scaled down to fit 8 B x n per tree of every
                                    graph into half of the device's memory                */
    int32_t walkers_per_tree;    /* 0 = automatic (teams of 64, fewer for graphs under
                                    1024 nodes); 1 = one walker per tree; else a power of
                                    two up to 64                                          */
    uint64_t max_steps_per_tree; /* guard; 0 = 2^20 + 4096 n                              */
    uint32_t graph_index_base;   /* Philox graph word of graphs[0]; graph g uses base + g */
    uint32_t strata;             /* 0 or 1: independent draws.  L >= 2 (at most 2^31):
                                    stratified stack entries, a variance reduction at equal
                                    trees (future work of the Conclusion: more efficient
                                    sampling).  The k-th departure from u takes, in sample i,
                                    stratum sigma_(u,k)(i) of L equal strata of its 64-bit
                                    word, sigma_(u,k) a permutation of 0 .. L-1 drawn for
                                    that stack entry (Latin hypercube over the samples); its
                                    own Philox word places it inside the stratum.  Each tree
                                    is still an exact Wilson tree and the visit totals stay
                                    unbiased; over samples 0 .. L-1 the variance of their
                                    mean can only drop (measured: to 0.5-0.8 of independent
                                    draws).  The call's samples must lie in [0, L); calls
                                    that cover [0, L) in pieces add up to the same totals.
                                    The squared totals then overstate the variance of the
                                    mean.  Definition: stratified_word in csrc/device.hpp  */
    const int32_t* roots;        /* DEVICE int32 [num_roots]: a root set S instead of one root
                                    (single graph, root = -1): every tree is a spanning forest
                                    rooted at S, i.e. Algorithm 3 with InTree = S at the start
                                    of each sample.  Ids must be distinct and in [0, n); a
                                    violation is reported by rwc_workspace_status (the
                                    outputs are then meaningless).  On a CSR with several
                                    components S must meet each one; a miss is reported the
                                    same way, as RWC_ERR_DISCONNECTED.  NULL when
                                    num_roots = 0                                            */
    int32_t num_roots;           /* 0: one root (`root`); else 1 .. n - 1                    */
    int32_t reserved2;
    const int32_t* walkers_per_graph; /* HOST [num_graphs] or NULL: walkers per tree of each
                                    graph (1 or a power of two up to 64), overriding
                                    walkers_per_tree (rwc_autotune_batch picks them)       */
} rwc_sample_params;

typedef struct rwc_sample_outputs {
    uint64_t* counts;            /* [sum n_g] visit totals: entry u of graph g is the sum
                                    over the trees of Algorithm 3's visit count of u (t~_u
                                    times l).  Graph g starts at offset sum_{h<g} n_h.     */
    uint64_t* counts_sq;         /* [sum n_g] sum of squared per-tree visits, or NULL     */
    uint64_t* total_steps;       /* [num_graphs] RandomNeighbor calls, or NULL            */
    uint64_t* tree_hash;         /* [num_graphs * num_samples] per-tree checksum
                                    sum_{u != root} splitmix64(u * 2^32 + parent(u)) mod 2^64,
                                    or NULL                                               */
    int32_t* parents;            /* [ndump * n] parent of each node in the dumped trees,
                                    -1 at the root (single graph only), or NULL           */
    const int64_t* dump_samples; /* HOST array [ndump] of absolute sample indices         */
    int32_t ndump;               /* at most 64                                            */
    int32_t reserved;
    float* timing_ms;            /* HOST [2] or NULL: device time of the walk kernels and of
                                    the reduction kernels, summed over batches (hipEvents on
                                    `stream`; not available with RWC_SAMPLE_GRAPH_CAPTURE) */
    int32_t* plan;               /* HOST [8] or NULL, as used for graph 0: walkers per tree,
                                    trees in flight, number of batches, walk kernel (0 one
                                    walker per tree, 1 walker teams, 2 walker teams with the
                                    LDS path ring), team starts (0 shared, 1 spread), start
                                    order (0 ascending ids, 1 breadth-first), hipGraph
                                    (-1 none, 0 captured by this call, 1 a cached graph
                                    replayed), graphs with LDS-resident trees.  The walk
                                    kernel is 3 (4 with the path ring) when graph 0's trees
                                    live in LDS                                           */
} rwc_sample_outputs;

/* Workspace for rwc_sample_forests with these graphs and parameters. */
int rwc_sample_forests_workspace(const rwc_csr* graphs, int32_t num_graphs,
                                 const rwc_sample_params* p, size_t* bytes);

/* Samples p->num_samples rooted spanning trees of each graph with Wilson's algorithm
 * (Section 5; Algorithm 3 with its visit counting) and accumulates per-node visit totals.
 * The k-th departure from node u in sample i of graph g takes RandomNeighbor(u) from
 * Philox4x32-10 on the counter (k, u, i, g) under key `seed`, so the forest is a fixed
 * function of (graph, seed, sample index) whatever the launch shape, the number of trees in
 * flight, the walkers per tree, or plain versus batched launches.
 *   graphs   HOST array [num_graphs] of graphs from rwc_build_csr
 * Stream-ordered: the call enqueues its work on `stream` and returns without waiting for it
 * (the small host arrays it reads, graphs, params, outputs and dump_samples, may be reused as
 * soon as it returns).  Device-side errors (RWC_ERR_STEP_LIMIT, RWC_ERR_COUNT_OVERFLOW, a bad
 * root set) are left in the workspace and returned by rwc_workspace_status.  Exception: with
 * out->timing_ms the call waits for its work (the timings need it) and returns the device
 * status itself.
 * On a stream that is being captured into a caller's hipGraph, the workspace must have been
 * prepared by rwc_sample_prepare with the same graphs, parameters (other than seed and
 * sample_begin) and workspace; the call then only launches kernels. */
int rwc_sample_forests(const rwc_csr* graphs, int32_t num_graphs, const rwc_sample_params* p,
                       const rwc_sample_outputs* out, void* ws, size_t ws_bytes, void* stream);

/* Writes the device-side argument tables that rwc_sample_forests reads (graph arguments, node
 * offsets, work items) into the workspace, for calls made while `stream` is being captured
 * into a hipGraph (a capture cannot hold the host-to-device copies).  The same arguments as
 * rwc_sample_forests; seed and sample_begin may differ in the captured calls.  Synchronises
 * `stream`.  The workspace must not be changed between this call and the replays. */
int rwc_sample_prepare(const rwc_csr* graphs, int32_t num_graphs, const rwc_sample_params* p, void* ws,
                       size_t ws_bytes, void* stream);

/* Frees the hipGraphs kept for RWC_SAMPLE_GRAPH_CAPTURE (waiting for their last launches). */
void rwc_release_cached_graphs(void);

/* Synchronises `stream` and returns the device-side outcome of the last stream-ordered call
 * that used the workspace `ws` (a sampling, estimate or adjoint workspace): RWC_OK or the
 * rwc_status its kernels reported.  RWC_ERR_INVALID_ARG if the workspace was never used. */
int rwc_workspace_status(const void* ws, void* stream);

/* Synchronises `stream` and stores the solver iterations run by the last estimate call on
 * the workspace `ws` in *iters. */
int rwc_workspace_iterations(const void* ws, int32_t* iters, void* stream);

/* ---- Trap walks: the estimator that FastWalk improves on (Lemma 5.1) -------------------- */
typedef struct rwc_trap_params {
    uint64_t seed;                /* Philox key (seed mod 2^32, seed >> 32)                  */
    int64_t walk_begin;           /* index of the first walk from each start node            */
    int64_t num_walks;            /* walks per start node (l)                                */
    int32_t trap;                 /* -1: the pivot                                           */
    uint32_t graph_index;         /* the walks use the Philox graph word graph_index ^ 2^31  */
    uint64_t max_steps_per_walk;  /* guard; 0 = 2^20 + 4096 n                                */
} rwc_trap_params;

int rwc_sample_trap_walks_workspace(const rwc_csr* g, const rwc_trap_params* p, size_t* bytes);

/* Lemma 5.1: (calL_v^{-1})_uu is the expected number of visits to u of a random walk from u
 * that stops at the trap v.  From every node u != v, num_walks independent walks (indices
 * walk_begin .. walk_begin + num_walks - 1) run until they reach v, each counting its visits
 * to u (the start included); walk i from u takes its s-th step by RandomNeighbor (the rule of
 * rwc_sample_forests) with Philox4x32-10 on the counter (s, u, i, graph_index ^ 2^31).
 *   counts_dev       uint64 [n] per start node, the sum of its walks' visit counts (0 at v):
 *                    rwc_estimate(counts, l = num_walks) assembles RWC from them exactly as
 *                    from the Wilson forests' visit totals
 *   counts_sq_dev    uint64 [n] sum of the squared counts, or NULL
 *   total_steps_dev  uint64 [1] RandomNeighbor calls, or NULL
 * Stream-ordered; a walk longer than max_steps_per_walk is reported by rwc_workspace_status
 * (RWC_ERR_STEP_LIMIT). */
int rwc_sample_trap_walks(const rwc_csr* g, const rwc_trap_params* p, uint64_t* counts_dev,
                          uint64_t* counts_sq_dev, uint64_t* total_steps_dev, void* ws, size_t ws_bytes,
                          void* stream);

typedef struct rwc_tune_result {
    int32_t walkers_per_tree;    /* the winning walkers per tree                            */
    int32_t trees_in_flight;     /* the winning trees in flight                              */
    double steps_per_s;          /* walk steps per second of the winning probe               */
    int32_t candidates;          /* probes run (0 when served from the cache)                */
    int32_t cached;              /* 1 if the result came from the per-process cache          */
    uint32_t flags;              /* schedule flags of the winner: for walker teams one of
                                    each pair PATH_RING / NO_PATH_RING, SHARED_STARTS /
                                    SPREAD_STARTS, ID_STARTS / BFS_STARTS, or 0 when the
                                    automatic schedule won; 0 for one walker per tree       */
    int32_t reserved;
} rwc_tune_result;

/* Workspace for rwc_autotune_sampler: room for the largest candidate whose slot state fits
 * `budget_bytes`, plus one graph's counts. */
int rwc_autotune_workspace(const rwc_csr* g, const rwc_sample_params* p, int64_t budget_bytes,
                           size_t* bytes);

/* Chooses walkers_per_tree, trees_in_flight and the team schedule for sampling `g` with
 * parameters `p` by timing one batch of each candidate on the real sample range: first 1, 8,
 * 16, 32 or 64 walkers per tree with one or two device-fulls of resident waves or all trees in
 * flight (slot state within budget_bytes) under the automatic schedule, then, for a winning
 * team, all eight combinations of path ring, start sharing and start order.  Caches the winner
 * per graph class (log2 n, mean degree, weighted, log2 l) for the process.  The forest does not
 * depend on the choice, only the speed.  Synchronises `stream`. */
int rwc_autotune_sampler(const rwc_csr* g, const rwc_sample_params* p, int64_t budget_bytes,
                         rwc_tune_result* out, void* ws, size_t ws_bytes, void* stream);

typedef struct rwc_batch_tune_result {
    int32_t walkers_mesh;        /* walkers per tree for the graphs with spread starts (pivot
                                    eccentricity above 32: mesh-like, long walks)            */
    int32_t walkers_other;       /* walkers per tree for the other graphs                    */
    uint32_t flags;              /* the winner's schedule flags: one of each pair PATH_RING /
                                    NO_PATH_RING, ID_STARTS / BFS_STARTS, and NO_LDS_STATE or
                                    0 (LDS-resident trees where they fit)                     */
    int32_t candidates;          /* probes run (0 when served from the cache)                */
    double steps_per_s;          /* walk steps per second of the winning probe               */
    int32_t probe_samples;       /* trees per graph in each probe                            */
    int32_t cached;              /* 1 if the result came from the per-process cache          */
} rwc_batch_tune_result;

/* Workspace for rwc_autotune_batch with these graphs and parameters. */
int rwc_autotune_batch_workspace(const rwc_csr* graphs, int32_t num_graphs, const rwc_sample_params* p,
                                 size_t* bytes);

/* Autotuning of a multi-graph call (the batched persistent launch): times probes of the real
 * sampler on all graphs at once, each with min(l, max(64, l / 8)) trees per graph from the
 * call's sample range: first the walkers per tree of the mesh-like graphs and of the others
 * (16, 32 or 64 each, nine probes) under the automatic schedule, then, for the winning pair,
 * the path ring on or off, ascending or breadth-first start order, and LDS-resident trees on
 * or off (eight probes).  Use the result with p->walkers_per_graph (mesh-like graphs, pivot
 * eccentricity above 32, take walkers_mesh) and p->flags |= flags.  Cached per (number of
 * graphs, their total nodes and entries, probe size) for the process.  The forest does not
 * depend on the choice, only the speed.  Synchronises `stream`. */
int rwc_autotune_batch(const rwc_csr* graphs, int32_t num_graphs, const rwc_sample_params* p,
                       rwc_batch_tune_result* out, void* ws, size_t ws_bytes, void* stream);

/* Forgets every cached tuning result. */
void rwc_autotune_clear_cache(void);

typedef struct rwc_solve_params {
    double tol;        /* relative residual of the pivot solve; 0 = 1e-12                 */
    int32_t max_iter;  /* 0 = 20000 (host-checked mode); stream-ordered mode: 1..4096,
                          required                                                        */
    int32_t check_every; /* iterations between host convergence checks; 0 = 16.  A negative
                          value selects stream-ordered mode: max_iter iterations are
                          enqueued at once and the solve stops on the device when the
                          residual meets tol (the same iterations a host-checked solve
                          runs, so the results are identical); the call then returns
                          without waiting, *iters is set to -1, and convergence is
                          reported by rwc_workspace_status (RWC_ERR_NOT_CONVERGED), the
                          count by rwc_workspace_iterations.  This mode can be captured
                          into a hipGraph.                                                 */
} rwc_solve_params;

int rwc_estimate_workspace(const rwc_csr* g, size_t* bytes);

/* AppRWC (Algorithm 1) fed by the FastWalk estimate t~ = counts / l (Algorithm 3, last line).
 * The pivot column of Algorithm 1 is obtained from the hitting times h_u = H_{u,pivot},
 * which solve the grounded system L_v h = d_{-v} (Jacobi-preconditioned CG in FP64);
 * Eq. (3) then reads RWC_u = vol t~_u / d_u - 2 h_u + RWC_v with RWC_v = sum_u d_u h_u / vol.
 *   counts_dev     uint64 [n] visit totals from rwc_sample_forests (this graph's slice)
 *   counts_sq_dev  uint64 [n] or NULL (needed for stderr_dev)
 *   l              number of trees behind counts
 *   rwc_dev        double [n] output RWC
 *   hit_dev        double [n] output hitting times to the pivot, or NULL
 *   stderr_dev     double [n] output standard error of rwc from the sample variance, or NULL
 *   iters          HOST int32 output: CG iterations used, or NULL
 * Host-checked mode synchronises `stream` (every check_every iterations and at the end) and
 * returns RWC_ERR_NOT_CONVERGED itself; stream-ordered mode (sp->check_every < 0) does not. */
int rwc_estimate(const rwc_csr* g, const uint64_t* counts_dev, const uint64_t* counts_sq_dev,
                 int64_t l, const rwc_solve_params* sp, double* rwc_dev, double* hit_dev,
                 double* stderr_dev, int32_t* iters, void* ws, size_t ws_bytes, void* stream);

/* rwc_estimate without a workspace, for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it).  The same
 * arguments, kernels and results as rwc_estimate in host-checked mode, over a fixed 128 MiB
 * device array inside the library (one per GPU the library runs on, held until the process
 * ends), which fits graphs of up to about 3.35 million nodes.  Calls no allocating routine.
 * RWC_ERR_TOO_LARGE if the graph needs more than the array holds; RWC_ERR_INVALID_ARG for the
 * stream-ordered mode (sp->check_every < 0).  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other threads, other streams) race and must be serialised by
 * the caller.  Synchronises `stream`. */
int rwc_estimate_static(const rwc_csr* g, const uint64_t* counts_dev, const uint64_t* counts_sq_dev,
                        int64_t l, const rwc_solve_params* sp, double* rwc_dev, double* hit_dev,
                        double* stderr_dev, int32_t* iters, void* stream);

int rwc_estimate_group_workspace(const rwc_csr* g, size_t* bytes);

/* Random walk centrality of a group of nodes (the generalisation named in the paper's
 * Conclusion): the group RWC H_S = sum_u pi_u H_{u,S} of a root set S (hitting time to the
 * set), and for every node u the estimate of H_{S + u} from spanning forests rooted at S
 * (rwc_sample_forests with p->roots = S).  With h the hitting times to S (the system grounded
 * at S, solved as in rwc_estimate) and t~_u = counts_u / l, which estimates d_u (L_S^-1)_uu as
 * Lemma 5.2 does for one root, removing u from the grounded system is a rank-one update:
 *   H_{S + u} = H_S - d_u h_u^2 / (vol t~_u)   (u not in S),   H_{S + u} = H_S (u in S).
 *   roots_dev      int32 [num_roots] the set S (distinct ids in [0, n), 1 <= num_roots < n)
 *   counts_dev     uint64 [n] visit totals of l forests rooted at S
 *   group_rwc_dev  double [1] output H_S
 *   marginal_dev   double [n] output H_{S + u}
 *   hit_dev        double [n] output hitting times to S, or NULL
 * Modes and synchronisation as rwc_estimate; a bad root set is RWC_ERR_INVALID_ARG or
 * RWC_ERR_NODE_RANGE (host-checked mode), or reported by rwc_workspace_status.  On a CSR with
 * several components S must meet each one (else RWC_ERR_DISCONNECTED, reported by
 * rwc_workspace_status). */
int rwc_estimate_group(const rwc_csr* g, const int32_t* roots_dev, int32_t num_roots,
                       const uint64_t* counts_dev, int64_t l, const rwc_solve_params* sp,
                       double* group_rwc_dev, double* marginal_dev, double* hit_dev, int32_t* iters,
                       void* ws, size_t ws_bytes, void* stream);

typedef struct rwc_backward_params {
    int32_t k;           /* Rademacher probes per sign class of g; 0 = exact (one column per
                            nonzero of g)                                                 */
    int32_t max_iter;    /* 0 = 20000                                                      */
    uint64_t seed;       /* probe key: the sign of probe i at node u is bit 0 of word 0 of
                            Philox4x32-10 on the counter (i, u, 0, 2^32 - 1); probes of the
                            negative class are numbered k .. 2k-1                          */
    double tol;          /* relative residual of every solve column; 0 = 1e-10            */
    int32_t check_every; /* iterations between host convergence checks; 0 = 16.  Iterations
                            launched past the last column's convergence return at once,
                            so the result and `iters` do not depend on it              */
    int32_t max_support; /* exact mode (k = 0): the most nonzeros g may have (the workspace
                            holds 2 + max_support solve columns); ignored when k > 0       */
} rwc_backward_params;

/* Workspace for rwc_backward: sized for 2 + 2k solve columns (k > 0: both sign classes of g)
 * or 2 + bp->max_support (exact mode).  RWC_ERR_INVALID_ARG for k < 0 or an exact-mode
 * max_support outside [1, n]; RWC_ERR_TOO_LARGE for more than 2^24 solve columns. */
int rwc_backward_workspace(const rwc_csr* g, const rwc_backward_params* bp, size_t* bytes);

/* Gradient of l(w) = sum_j g_j RWC_j (exact RWC, Eq. (2)) with respect to every edge weight.
 * The paper does not differentiate RWC; this is the adjoint of its quantity, with the
 * derivative of L^+ through the incidence form L = B^T B of Section 2.2:
 *   dl/dw_e = 2 trGL - vol Q_e + 2 D_A D_B - 2 S_A + G ((2 S_B - D_B^2)/vol - 2 d^T B/vol^2)
 * A = L^+ g, B = L^+ d, G = sum g, trGL = sum_j g_j L^+_jj, Q_e = sum_j g_j (L^+ b_e)_j^2,
 * D_X = X_a - X_b, S_X = X_a + X_b for e = (a, b).  Q_e and trGL are exact (k = 0: one solve
 * column per nonzero of g) or a Johnson-Lindenstrauss / Hutchinson sketch with k probes per
 * sign class of g.  All solves run together as one batched Jacobi-preconditioned CG on the
 * grounded Laplacian (FP32 search directions, FP64 iterate, residual and dot products).
 *   grad_rwc_dev  double [n] the vector g (device); its support and signs are found on the
 *                 device.  RWC_ERR_INVALID_ARG if it holds a value that is not finite or
 *                 (exact mode) more than max_support nonzeros; if it is zero everywhere the
 *                 gradient is zero
 *   grad_w_dev    double [m] output in input-edge order (device)
 *   iters         HOST int32 output: CG iterations run (up to the last column's
 *                 convergence), or NULL
 * Synchronises `stream` (it reads back the support counts, then checks convergence every
 * check_every iterations). */
int rwc_backward(const rwc_csr* g, const double* grad_rwc_dev, const rwc_backward_params* bp,
                 double* grad_w_dev, int32_t* iters, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * FastChol (Section 4, Algorithm 2): the matrix-factorisation estimate of diag(calL_v^{-1}),
 * the second of the paper's two algorithms, on the GPU.
 *
 * 1. IChol(calL_v, delta) (Lemma 4.1): incomplete Cholesky of the grounded normalised
 *    Laplacian (pivot v removed, columns in ascending input id), left-looking; an off-diagonal
 *    entry x of column j is kept when |x| >= delta * ||calL_v(j:N, j)||_1 (the threshold rule of
 *    the ICT variant of MATLAB's ichol, which the paper's experiments use with delta = 1e-4).
 * 2. The sparse approximate inverse S~ of the factor, right to left (Lemma 4.3's recursion
 *    over a sliding window of w_u = min(floor(w_s (1 + d_u / d_max)), N) later columns), each
 *    column of more than zeta nonzeros cut to the shortest prefix, by decreasing magnitude,
 *    whose dropped tail has 1-norm <= eps_p times the column's (Algorithm 2's sparsification);
 *    tau~_u = ||S~(:, u)||^2 (Section 4: (calL_v^{-1})_uu ~ ||R^{-1} e_u||^2).
 * Both are chains of dependent columns; one wave runs each, column by column, in the serial
 * algorithm's order of floating-point operations.  Feed tau~ to rwc_estimate_diag for RWC.
 * ------------------------------------------------------------------------------------- */
/* How rwc_fastchol factors calL_v; both give the same factor bit for bit.
 *   RWC_FASTCHOL_DENSE: right-looking on the packed lower triangle of the (n-1) x (n-1) matrix
 *     ((n-1) n / 2 doubles) in the workspace, one
 *     launch per column, the column's updates spread over the GPU (n - 1 <= 2^20);
 *   RWC_FASTCHOL_CHAIN: left-looking on one wave, sparse throughout (any n; a column may reach
 *     at most 4096 kept entries);
 *   RWC_FASTCHOL_AUTO: DENSE while that triangle is at most 32 GiB ((n-1) <= 92681), else CHAIN. */
#define RWC_FASTCHOL_AUTO 0
#define RWC_FASTCHOL_CHAIN 1
#define RWC_FASTCHOL_DENSE 2

typedef struct rwc_fastchol_params {
    double droptol;            /* IChol drop tolerance delta (>= 0; the paper uses 1e-4)         */
    double window;             /* base window width w_s (>= 1)                                   */
    double eps_p;              /* sparsification tolerance (>= 0)                                */
    int32_t zeta;              /* columns of at most zeta nonzeros are kept whole (>= 0)         */
    int32_t method;            /* RWC_FASTCHOL_AUTO, _CHAIN or _DENSE                            */
    int64_t factor_capacity;   /* entries of the factor the workspace holds (>= n - 1); a factor
                                  that needs more stops with RWC_ERR_TOO_LARGE                */
    int64_t inverse_capacity;  /* entries of S~ the workspace holds                          */
} rwc_fastchol_params;

int rwc_fastchol_workspace(const rwc_csr* g, const rwc_fastchol_params* p, size_t* bytes);

/* tau_dev: double [n] output by input id (0 at the pivot).  Stream-ordered: the call enqueues
 * its kernels (five for CHAIN, n + 6 for DENSE; the inverse is one workgroup) and returns;
 * rwc_workspace_status reports RWC_ERR_TOO_LARGE (a pool, or a column's 4096-entry ordering
 * buffer, was too small) or RWC_ERR_BREAKDOWN (a non-positive pivot), after which tau_dev is
 * meaningless.  RWC_ERR_INVALID_ARG for an unknown method, RWC_ERR_TOO_LARGE for DENSE past
 * 2^20 columns. */
int rwc_fastchol(const rwc_csr* g, const rwc_fastchol_params* p, double* tau_dev, void* ws, size_t ws_bytes,
                 void* stream);

/* Entries of the factor and of S~ the last rwc_fastchol on `ws` produced (synchronises). */
int rwc_fastchol_sizes(const void* ws, int64_t* factor_entries, int64_t* inverse_entries, void* stream);

/* AppRWC (Algorithm 1) from an estimate of diag(calL_v^{-1}) itself (FastChol's tau~) instead
 * of visit totals: rwc_estimate with t~ = diag_dev (double [n] by input id; the pivot's entry is
 * not read).  Same workspace, parameters, outputs and synchronisation as rwc_estimate. */
int rwc_estimate_diag(const rwc_csr* g, const double* diag_dev, const rwc_solve_params* sp, double* rwc_dev,
                      double* hit_dev, int32_t* iters, void* ws, size_t ws_bytes, void* stream);

const char* rwc_status_string(int status);
/* Copies the calling thread's last error detail into buf (NUL-terminated); returns its
 * length. */
int rwc_last_error(char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* RWC_H */
