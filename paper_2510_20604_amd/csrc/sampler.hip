// rwc_sample_forests: Wilson's algorithm (Section 5, Algorithm 3) on the GPU, many trees at
// once, with the visit counting of Algorithm 3 reduced into per-node totals.
//
// Layout.  Each graph g keeps T tree slots; slot t holds one 64-bit state word per node
// (state[t * n_g + u], see device.hpp) -- the InTree flag, Next[u] and the departure count
// of u in the slot's current tree.  A batch runs T trees (one per slot) to completion, then a
// reduction pass folds the per-tree departure counts into the per-node totals, writes the
// requested parent dumps and resets the slots for the next batch.
//
// Two kernels (walk.hpp).  wilson_walk: one lane grows one tree, running Algorithm 3's three loops --
// pick the next start node that is not yet in the tree, walk until the tree is hit, retrace
// the loop-erased path -- as one flat state machine, so every iteration of the wave does one
// step of some lane's work instead of parking lanes that finished a phase early.
// wilson_team: W lanes of one wave grow one tree together (below); used for large graphs,
// whose per-tree state limits how many trees can be in flight.
//
// RandomNeighbor(u) at the k-th departure from u in sample i of graph word g is
// Philox4x32-10((k, u, i, g), seed).  A node's successive choices are therefore fixed in
// advance, which makes the tree and every count independent of the order in which walks are
// run (cycle popping), so results match the serial order of Algorithm 3 exactly.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "roots.hpp"
#include "device.hpp"
#include "walk.hpp"

namespace rwc {

int team_resident_waves(bool ring) {
    static std::atomic<int> cached[2] = {{0}, {0}};   // waves per CU (a property of the code object)
    int per_cu = cached[ring ? 1 : 0].load();
    if (per_cu == 0) {
        const hipError_t e = ring ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wilson_team<true>, kWave, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wilson_team<false>, kWave, 0);
        if (e != hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        } else {
            cached[ring ? 1 : 0].store(per_cu);
        }
    }
    return per_cu * device_cu_count();
}

namespace {

// Start positions for a team: spread or shared as asked, otherwise spread for graphs whose
// pivot eccentricity marks them as long-walk (mesh-like) graphs.  On such graphs consecutive starts lie next to
// each other and a team's walkers keep blocking one another; on small-world graphs
// consecutive starts keep the team inside a hot region of the graph.
constexpr int32_t kLongWalkDepth = 32;

bool spread_starts(const rwc_csr& g, uint32_t flags) {
    if (flags & RWC_SAMPLE_SPREAD_STARTS) return true;
    if (flags & RWC_SAMPLE_SHARED_STARTS) return false;
    return g.bfs_depth > kLongWalkDepth;
}

using LdsKernel = void (*)(const GraphArgs*, const Item*, int32_t, uint32_t*, int64_t, int64_t, uint64_t,
                           const int64_t*, uint64_t*, uint64_t*, int32_t*, DumpArgs, uint64_t*, uint64_t*, uint32_t*);
using WalkKernel = void (*)(const GraphArgs*, const Item*, int32_t, uint32_t*, int32_t, int64_t, int64_t, uint64_t,
                            uint64_t*, uint64_t*, uint32_t*);

__device__ __forceinline__ int32_t graph_of(const int64_t* __restrict__ node_off, int32_t G, int64_t gx) {
    int32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (node_off[mid] <= gx)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool is_root(const GraphArgs& A, int64_t x) {
    return A.rootmask ? ((A.rootmask[x >> 5] >> (x & 31)) & 1u) != 0 : x == A.root;
}

// Sets every slot of every graph to the fresh state (the roots in the tree, all else zero).
__global__ void init_state(const GraphArgs* __restrict__ graphs, const int64_t* __restrict__ node_off, int32_t G,
                           int64_t total_nodes) {
    for (int64_t gx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; gx < total_nodes;
         gx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t g = graph_of(node_off, G, gx);
        const GraphArgs A = graphs[g];
        const int64_t x = gx - node_off[g];
        const uint64_t v = is_root(A, x) ? kInTree : 0ull;
        for (int32_t t = 0; t < A.T; ++t) A.state[static_cast<int64_t>(t) * A.stride + x] = v;
    }
}

// First kernel of a call: clears the outputs (unless accumulating), the root bitmap and the
// work queue, and starts the workspace header.
__global__ void zero_outputs(uint64_t* counts, uint64_t* counts_sq, int64_t total_nodes, uint64_t* total_steps,
                             int32_t G, WsHeader* header, uint32_t* queue, uint32_t* rootmask, int64_t mask_words) {
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = tid; i < total_nodes; i += stride) {
        if (counts) counts[i] = 0;
        if (counts_sq) counts_sq[i] = 0;
    }
    for (int64_t i = tid; i < mask_words; i += stride) rootmask[i] = 0u;
    for (int64_t i = tid; i < G; i += stride)
        if (total_steps) total_steps[i] = 0;
    if (tid == 0) {
        header_begin(header);
        queue[0] = 0;
        queue[1] = 0;
    }
}

// Root set of a single graph: one bit per root id.  Ids out of range or listed twice are
// reported through the header (the trees of such a call are not sampled: init_state and the
// walk still run, but the status tells the caller to discard the outputs).
__global__ void build_rootmask(const int32_t* __restrict__ roots, int32_t nroots, int32_t n,
                               const int32_t* __restrict__ node_index, uint32_t* __restrict__ rootmask,
                               WsHeader* header) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nroots) return;
    const int32_t id = roots[i];
    if (id < 0 || id >= n) {
        atomicOr(&header->status, static_cast<uint32_t>(kErrNodeRange));
        return;
    }
    const int32_t r = node_index[id];
    const uint32_t bit = 1u << (r & 31);
    const uint32_t old = atomicOr(&rootmask[r >> 5], bit);
    if (old & bit) atomicOr(&header->status, static_cast<uint32_t>(kErrDupRoot));
}

__global__ void reset_queue(uint32_t* queue) { *queue = 0; }

// An explicit root arrives as an input id; its internal index is known on the device only.
__global__ void resolve_root(GraphArgs* graphs, const int32_t* __restrict__ node_index, int32_t root_id) {
    graphs[0].root = node_index[root_id];
}

// Folds the departure counts of batch `batch` into the per-node totals, writes the parent
// dumps of this batch and, unless it is the last batch, resets the slots for the next one.  Thread per node, loop over slots: the reads and
// writes of consecutive threads are consecutive words of one slot.
__global__ void reduce_batch(const GraphArgs* __restrict__ graphs, const int64_t* __restrict__ node_off, int32_t G,
                             int64_t total_nodes, int32_t batch, int64_t l, bool reset,
                             uint64_t* __restrict__ counts, uint64_t* __restrict__ counts_sq,
                             int32_t* __restrict__ parents, DumpArgs dumps) {
    for (int64_t gx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; gx < total_nodes;
         gx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t g = graph_of(node_off, G, gx);
        const GraphArgs A = graphs[g];
        const int64_t x = gx - node_off[g];
        const int64_t first = static_cast<int64_t>(batch) * A.T;
        const int32_t used = static_cast<int32_t>(first >= l ? 0 : ((l - first) < A.T ? (l - first) : A.T));
        const bool root = is_root(A, x);
        const int64_t id = A.node_id[x];   // outputs are indexed by input id
        for (int d = 0; d < dumps.count; ++d) {
            const uint64_t w = A.state[static_cast<int64_t>(dumps.slot[d]) * A.stride + x];
            parents[static_cast<int64_t>(dumps.out[d]) * A.n + id] = root ? -1 : A.node_id[st_next(w)];
        }
        const uint64_t fresh = root ? kInTree : 0ull;
        uint64_t c1 = 0, c2 = 0;
        int32_t t = 0;
        for (; t + 4 <= used; t += 4) {
            uint64_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = A.state[static_cast<int64_t>(t + q) * A.stride + x];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t c = st_cnt(w[q]);
                c1 += c;
                c2 += square_count(c);
                if (reset) A.state[static_cast<int64_t>(t + q) * A.stride + x] = fresh;
            }
        }
        for (; t < used; ++t) {
            const uint32_t c = st_cnt(A.state[static_cast<int64_t>(t) * A.stride + x]);
            c1 += c;
            c2 += square_count(c);
            if (reset) A.state[static_cast<int64_t>(t) * A.stride + x] = fresh;
        }
        if (counts) counts[node_off[g] + id] += c1;
        if (counts_sq) counts_sq[node_off[g] + id] += c2;
    }
}

// ---------------------------------------------------------------------- planning ------
struct Plan {
    std::vector<int32_t> W, T, S;     // per graph: walkers per tree, tree slots, trees per wave
    std::vector<int64_t> stride;      // per graph: words per slot
    std::vector<char> lds;            // per graph: its trees live in LDS (no slots in HBM)
    std::vector<int64_t> node_off;
    int64_t total_nodes = 0;
    int64_t lds_words = 0;            // dynamic LDS of the LDS-state kernel, in 8-byte words
    int32_t batches = 1;
    int32_t lds_graphs = 0;
    bool team = false;                // some graph uses more than one walker per tree
    bool hbm_team = false;            // some graph with HBM state uses walker teams
};

// LDS per wave for the state words of an LDS-resident graph's trees (64 / W trees of n
// words, n rounded up to 8): with the 8 KB of path ring and record copies, 56 KB per wave,
// two waves per compute unit at the largest size.
constexpr int64_t kLdsStateBytes = 48 * 1024;
constexpr int64_t kLdsMaxSamples = int64_t{1} << 24;

// Bytes of tree state the automatic plan may use: half of the device's memory (144 GB of the
// 288 GB of an MI355X), so that every tree of BA(10^6) x 10^4 (80 GB) or of R-MAT scale 23 x
// 5000 (133 GB) is in flight at once.  Total, not free, memory keeps the plan identical between
// the workspace query and the call that uses the workspace.
int64_t default_state_budget() {
    // cached per device: the total does not change, and a call made while a stream is being
    // captured should not query the runtime more than it must
    static std::mutex mu;
    static std::vector<int64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 96ll << 30;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (static_cast<int>(cache.size()) <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) {
            (void)hipGetLastError();
            return 96ll << 30;
        }
        cache[dev] = static_cast<int64_t>(total_b / 2);
    }
    return cache[dev];
}

// Walkers per tree when the caller leaves it open.  Full-wave teams, narrowed only for tiny
// graphs (at least 16 nodes per walker): on BA(10^6), 10^4 trees, 64 walkers beat 32, and on
// the 256-graph batch (BA and meshes, 10^3..10^5 nodes) 64 walkers for every graph beat widths
// growing with n by 3-5%.  Teams also beat one walker per tree on small problems, where one
// lane per tree leaves the device nearly empty and every step waits on its own memory
// latency: ER(1000) with 500 trees 9x, BA(3000) with 1000 trees 59x, a 2500-node grid 16x,
// and still with 200 000 trees of ER(1000) (1.6x at 32 walkers).
int auto_walkers(int64_t n) {
    int W = 64;
    while (W > 2 && W * 16 > n) W >>= 1;
    return W;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int make_plan(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p, Plan* plan) {
    plan->node_off.assign(G + 1, 0);
    plan->W.assign(G, 1);
    plan->T.assign(G, 1);
    plan->S.assign(G, kWave);
    plan->stride.assign(G, 0);
    plan->lds.assign(G, 0);
    for (int32_t g = 0; g < G; ++g) {
        if (graphs[g].n < 2 || !graphs[g].row_ptr || !graphs[g].col || !graphs[g].rec || !graphs[g].bfs_order)
            return fail(RWC_ERR_INVALID_ARG, "graph %d is not a built CSR", g);
        plan->node_off[g + 1] = plan->node_off[g] + graphs[g].n;
    }
    plan->total_nodes = plan->node_off[G];
    const int64_t l = p->num_samples;
    int64_t state_words = 0;
    // LDS-resident trees run in a launch of their own before the HBM-state walk.  Measured: a
    // single small graph gains (ER(1000), 2000 trees: walk 2.64 -> 1.84 ms), but in a batch that
    // also holds larger graphs the two launches cannot overlap and the LDS launch's tail idles
    // the device (256 mixed graphs: the batch autotuner picks HBM state), so a call uses LDS
    // state only when every graph's trees fit.
    bool all_fit = !(p->flags & RWC_SAMPLE_NO_LDS_STATE) && l <= kLdsMaxSamples;
    for (int32_t g = 0; g < G && all_fit; ++g) {
        const int Wg = p->walkers_per_graph ? p->walkers_per_graph[g]
                       : (p->walkers_per_tree > 0) ? p->walkers_per_tree : auto_walkers(graphs[g].n);
        all_fit = Wg > 1 && (kWave / Wg) * round_up(graphs[g].n, 8) * 8 <= kLdsStateBytes;
    }
    for (int32_t g = 0; g < G; ++g) {
        const int64_t n = graphs[g].n;
        const int W = p->walkers_per_graph ? p->walkers_per_graph[g]
                      : (p->walkers_per_tree > 0) ? p->walkers_per_tree : auto_walkers(n);
        const int S = kWave / W;
        int64_t T = p->trees_in_flight;
        if (T <= 0) {
            T = round_up(l, S);     // all trees at once; the state budget below may cut it
        }
        if (T > (1 << 30)) return fail(RWC_ERR_TOO_LARGE, "trees_in_flight too large");
        plan->W[g] = W;
        plan->S[g] = S;
        plan->T[g] = static_cast<int32_t>(T);
        plan->stride[g] = round_up(n, 8);
        plan->team = plan->team || W > 1;
        // trees in LDS when every graph's wave of trees fits (walker teams only), unless the
        // caller forbids it (the work items of LDS graphs list every block of samples, so very
        // long sample ranges keep their trees in HBM slots)
        if (all_fit) {
            plan->lds[g] = 1;
            plan->T[g] = 0;
            plan->lds_words = std::max<int64_t>(plan->lds_words, S * plan->stride[g]);
            ++plan->lds_graphs;
            continue;
        }
        plan->hbm_team = plan->hbm_team || W > 1;
        state_words += T * plan->stride[g];
    }
    const int64_t budget = (p->trees_in_flight <= 0) ? default_state_budget() : 0;
    if (p->trees_in_flight <= 0 && state_words * 8 > budget) {
        // shrink every graph's slots by the same factor to fit the automatic budget
        const double f = static_cast<double>(budget) / (8.0 * static_cast<double>(state_words));
        for (int32_t g = 0; g < G; ++g) {
            if (plan->lds[g]) continue;
            int64_t T = static_cast<int64_t>(plan->T[g] * f) / plan->S[g] * plan->S[g];
            plan->T[g] = static_cast<int32_t>(T < plan->S[g] ? plan->S[g] : T);
        }
    }
    int32_t batches = 1;
    for (int32_t g = 0; g < G; ++g) {
        if (plan->lds[g]) continue;   // all of an LDS graph's trees run in the first batch
        const int64_t b = (l + plan->T[g] - 1) / plan->T[g];
        batches = b > batches ? static_cast<int32_t>(b) : batches;
    }
    plan->batches = batches;
    return RWC_OK;
}

struct SampleLayout {
    WsHeader* header;
    std::vector<uint64_t*> state;
    GraphArgs* graphs;
    int64_t* node_off;
    Item* items;
    uint32_t* queue;
    uint32_t* rootmask;
    int64_t mask_words;
    uint32_t* cover;   // [n0] components holding a root (graphs of several components)
    size_t total;
};

// Work items of one batch of HBM-state graphs (a block of S tree slots each), then of the
// LDS-state graphs (a block of S samples each, all samples in one launch).
int64_t max_items(int32_t G, const Plan& plan, int64_t l) {
    int64_t k = 0;
    for (int32_t g = 0; g < G; ++g)
        k += plan.lds[g] ? (l + plan.S[g] - 1) / plan.S[g] : (plan.T[g] + plan.S[g] - 1) / plan.S[g];
    return k;
}

int64_t hbm_items(int32_t G, const Plan& plan) {
    int64_t k = 0;
    for (int32_t g = 0; g < G; ++g)
        if (!plan.lds[g]) k += (plan.T[g] + plan.S[g] - 1) / plan.S[g];
    return k;
}

SampleLayout carve_sample(void* ws, int32_t G, const Plan& plan, int32_t n0, int64_t l) {
    Carver c(ws);
    SampleLayout L{};
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.state.resize(G);
    for (int32_t g = 0; g < G; ++g) L.state[g] = c.take<uint64_t>(static_cast<size_t>(plan.T[g]) * plan.stride[g]);
    L.graphs = c.take<GraphArgs>(G);
    L.node_off = c.take<int64_t>(G + 1);
    L.items = c.take<Item>(max_items(G, plan, l));
    L.queue = c.take<uint32_t>(2);   // [0] HBM-state walk, [1] LDS-state walk
    // root bitmap of graph 0 (an explicit root set is for single-graph calls)
    L.mask_words = (static_cast<int64_t>(n0) + 31) / 32;
    L.rootmask = c.take<uint32_t>(L.mask_words);
    L.cover = c.take<uint32_t>(n0);
    L.total = c.used();
    return L;
}

// hipEvents bracketing the walk and reduction launches of every batch.
struct Timer {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    float walk_ms = 0.f, reduce_ms = 0.f;
    int init() {
        for (auto& e : ev) RWC_HIP(hipEventCreate(&e));
        return RWC_OK;
    }
    ~Timer() {   // teardown: failures here have nobody to report to
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

int validate(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p) {
    if (!graphs || !p || G < 1) return fail(RWC_ERR_INVALID_ARG, "graphs/params missing or num_graphs < 1");
    if (p->num_samples < 1) return fail(RWC_ERR_INVALID_ARG, "num_samples must be positive");
    if (p->sample_begin < 0 || p->num_samples > (1ll << 32) || p->sample_begin > (1ll << 32) - p->num_samples)
        return fail(RWC_ERR_INVALID_ARG, "sample indices must lie in [0, 2^32)");
    if (p->root >= 0 && G != 1) return fail(RWC_ERR_INVALID_ARG, "an explicit root needs a single graph");
    if (p->root >= graphs[0].n) return fail(RWC_ERR_INVALID_ARG, "root out of range");
    if (p->num_roots < 0 || (p->num_roots > 0 && (!p->roots || G != 1 || p->root >= 0)))
        return fail(RWC_ERR_INVALID_ARG, "a root set needs roots, a single graph and root = -1");
    if (p->num_roots >= graphs[0].n)
        return fail(RWC_ERR_INVALID_ARG, "the root set must leave at least one node outside it");
    // a disconnected graph needs a root set (one that meets every component, checked on the device)
    for (int32_t g = 0; g < G; ++g)
        if (graphs[g].components > 1 && p->num_roots == 0)
            return fail(RWC_ERR_DISCONNECTED, "graph %d has %d components: sample it with a root set that meets each",
                        g, graphs[g].components);
    const int W = p->walkers_per_tree;
    if (W < 0 || W > kWave || (W & (W - 1)) != 0)
        return fail(RWC_ERR_INVALID_ARG, "walkers_per_tree must be 0 (automatic) or a power of two up to 64");
    if (p->walkers_per_graph)
        for (int32_t g = 0; g < G; ++g) {
            const int w = p->walkers_per_graph[g];
            if (w < 1 || w > kWave || (w & (w - 1)) != 0)
                return fail(RWC_ERR_INVALID_ARG, "walkers_per_graph[%d] must be a power of two up to 64", g);
        }
    if (p->strata > (1u << 31)) return fail(RWC_ERR_INVALID_ARG, "strata must be at most 2^31");
    if (p->strata >= 2 && p->sample_begin + p->num_samples > static_cast<int64_t>(p->strata))
        return fail(RWC_ERR_INVALID_ARG, "stratified samples must lie in [0, strata)");
    if ((p->flags & RWC_SAMPLE_SPREAD_STARTS) && (p->flags & RWC_SAMPLE_SHARED_STARTS))
        return fail(RWC_ERR_INVALID_ARG, "spread and shared starts are exclusive");
    if ((p->flags & RWC_SAMPLE_PATH_RING) && (p->flags & RWC_SAMPLE_NO_PATH_RING))
        return fail(RWC_ERR_INVALID_ARG, "path ring and no path ring are exclusive");
    if ((p->flags & RWC_SAMPLE_BFS_STARTS) && (p->flags & RWC_SAMPLE_ID_STARTS))
        return fail(RWC_ERR_INVALID_ARG, "breadth-first and ascending starts are exclusive");
    return RWC_OK;
}

// The stratification constants of L samples (see stratified_word).
Strata make_strata(uint32_t L) {
    Strata S{0, 0, 0};
    if (L < 2) return S;
    uint32_t bits = 2;
    while ((1ull << bits) < L) ++bits;
    S.count = L;
    S.bits = bits;
    S.width = static_cast<uint64_t>((static_cast<unsigned __int128>(1) << 64) / L);
    return S;
}

// Everything a call derives on the host: the plan, the device tables (graph arguments, node
// offsets, work items) and the launch choices.
struct Setup {
    Plan plan;
    std::vector<GraphArgs> hg;
    std::vector<Item> items;
    bool ring = false, lds_ring = false;
    WalkKernel walk = nullptr;
    LdsKernel walk_lds = nullptr;
    int grid_persistent = 0;
    int32_t nit_hbm = 0, nit_lds = 0, grid_lds = 0;
    size_t lds_bytes = 0;
    SampleLayout L;
};

int make_setup(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p, void* ws, Setup* S) {
    Plan& plan = S->plan;
    RWC_CHECK(make_plan(graphs, G, p, &plan));
    S->L = carve_sample(ws, G, plan, graphs[0].n, p->num_samples);
    std::vector<GraphArgs>& hg = S->hg;
    hg.assign(G, GraphArgs{});
    bool any_spread = false, any_dense_weighted = false;
    for (int32_t g = 0; g < G; ++g) {
        const uint64_t n = static_cast<uint64_t>(graphs[g].n);
        // default step guard: far above the expected walk length of any graph we accept,
        // small enough that a runaway tree ends with an error instead of a hang
        uint64_t steps = p->max_steps_per_tree ? p->max_steps_per_tree : (1ull << 20) + 4096ull * n;
        // a team's iterations: every step, retrace, release and start check of a tree takes
        // at most one iteration of some walker, and waits end by cycle pops, which are looked
        // for every kPollEvery-th iteration
        if (plan.W[g] > 1) steps = static_cast<uint64_t>(kPollEvery) * steps + 8ull * n + 1024ull;
        hg[g].row_ptr = graphs[g].row_ptr;
        hg[g].col = graphs[g].col;
        hg[g].cdf = graphs[g].weighted ? graphs[g].cdf : nullptr;
        hg[g].rec = reinterpret_cast<const uint4*>(graphs[g].rec);
        hg[g].order = nullptr;   // set below, once every graph's start mode is known
        hg[g].state = S->L.state[g];
        hg[g].stride = plan.stride[g];
        hg[g].guard = steps;
        hg[g].rootmask = (g == 0 && p->num_roots > 0) ? S->L.rootmask : nullptr;
        hg[g].n = graphs[g].n;
        hg[g].node_id = graphs[g].node_id;
        hg[g].node_index = graphs[g].node_index;
        hg[g].root = (p->root >= 0) ? -1 : graphs[g].pivot_index;   // an explicit root: resolve_root
        hg[g].graph_word = p->graph_index_base + static_cast<uint32_t>(g);
        hg[g].T = plan.T[g];
        hg[g].W = plan.W[g];
        hg[g].spread = spread_starts(graphs[g], p->flags) ? 1 : 0;
        hg[g].strata = make_strata(p->strata);
        if (plan.W[g] > 1) {
            any_spread = any_spread || hg[g].spread;
            any_dense_weighted =
                any_dense_weighted || (graphs[g].cdf != nullptr && graphs[g].nnz > kRingMaxMeanDegree * graphs[g].n);
        }
    }
    // The ring saves the read of every buffered path node's word on attach and on loop
    // erasure, and shortens the iterations that do them.  Measured: needed on meshes (spread
    // starts); faster on unweighted graphs (BA(10^6) 5-8 %, BA(3*10^6) 10 %), on weighted BA
    // (BA(10^6), 4000 trees: 15 %) and whenever the call leaves much of the device idle
    // (R-MAT, 2000 trees: 23 %); slower on weighted graphs of high mean degree that fill the
    // device (weighted R-MAT scale 21-23, mean degree 22-25: 16-27 %).
    const int64_t resident = team_resident_waves(true);
    const int64_t l = p->num_samples;
    const bool fills = plan.hbm_team && 3 * hbm_items(G, plan) >= 2 * resident;
    // Start order, measured: breadth-first starts make batches of many meshes (spread starts)
    // a third faster (256 mixed graphs: 4.5 -> 3.0 s, their 128 grids alone 4.0 -> 3.1 s) but
    // every single graph slower, meshes included (a 25 k-node grid with 50 000 trees: 10 %, a
    // 97 k-node grid with 2000-20 000 trees: 5-15 %), and small-world graphs (shared starts)
    // by much more.  So they are taken for the meshes of calls with several graphs and a queue
    // of at least twice the resident waves.
    const bool queued = plan.team && G > 1 && max_items(G, plan, l) >= 2 * resident;
    for (int32_t g = 0; g < G; ++g) {
        const bool bfs = (p->flags & RWC_SAMPLE_BFS_STARTS) ||
                         (!(p->flags & RWC_SAMPLE_ID_STARTS) && queued && plan.W[g] > 1 && hg[g].spread);
        hg[g].order = bfs ? graphs[g].bfs_order : nullptr;
    }
    S->ring = (p->flags & RWC_SAMPLE_PATH_RING) ? true
              : (p->flags & RWC_SAMPLE_NO_PATH_RING) ? false
                                                      : (any_spread || !any_dense_weighted || !fills);
    // LDS-state trees: a buffered path node's word is an LDS access like any other, so the ring
    // saves little there; it is used only on request
    S->lds_ring = (p->flags & RWC_SAMPLE_PATH_RING) != 0;
    // Work items with the longest trees first: a tree's time grows with n / W.
    std::vector<int32_t> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return static_cast<int64_t>(graphs[a].n) * plan.W[b] > static_cast<int64_t>(graphs[b].n) * plan.W[a];
    });
    S->items.clear();
    S->items.reserve(max_items(G, plan, l));
    for (int32_t g : order)
        if (!plan.lds[g])
            for (int32_t s0 = 0; s0 < plan.T[g]; s0 += plan.S[g]) S->items.push_back(Item{g, s0});
    S->nit_hbm = static_cast<int32_t>(S->items.size());
    for (int32_t g : order)
        if (plan.lds[g])
            for (int64_t s0 = 0; s0 < l; s0 += plan.S[g]) S->items.push_back(Item{g, static_cast<int32_t>(s0)});
    S->nit_lds = static_cast<int32_t>(S->items.size()) - S->nit_hbm;
    const bool hbm_team = plan.hbm_team || (plan.team && S->nit_hbm == 0);
    const bool strat = p->strata >= 2;
    if (strat)
        S->walk = !hbm_team  ? static_cast<WalkKernel>(wilson_walk_strata)
                  : S->ring  ? static_cast<WalkKernel>(wilson_team_strata<true>)
                             : static_cast<WalkKernel>(wilson_team_strata<false>);
    else
        S->walk = !hbm_team  ? static_cast<WalkKernel>(wilson_walk)
                  : S->ring  ? static_cast<WalkKernel>(wilson_team<true>)
                             : static_cast<WalkKernel>(wilson_team<false>);
    if (p->flags & RWC_SAMPLE_PERSISTENT) {
        int per_cu = 0;
        RWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, S->walk, kWave, 0));
        if (per_cu < 1) per_cu = 1;
        S->grid_persistent = per_cu * device_cu_count();
    }
    if (S->nit_lds > 0) {
        if (strat)
            S->walk_lds = S->lds_ring ? static_cast<LdsKernel>(wilson_team_lds_strata<true>)
                                      : static_cast<LdsKernel>(wilson_team_lds_strata<false>);
        else
            S->walk_lds = S->lds_ring ? static_cast<LdsKernel>(wilson_team_lds<true>)
                                      : static_cast<LdsKernel>(wilson_team_lds<false>);
        S->lds_bytes = static_cast<size_t>(plan.lds_words) * 8;
        int per_cu = 0;
        RWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, S->walk_lds, kWave, S->lds_bytes));
        if (per_cu < 1) per_cu = 1;
        const int64_t grid = static_cast<int64_t>(per_cu) * device_cu_count();
        S->grid_lds = static_cast<int32_t>(grid < S->nit_lds ? grid : S->nit_lds);
    }
    return RWC_OK;
}

int upload_tables(const Setup& S, int32_t G, hipStream_t s) {
    RWC_HIP(hipMemcpyAsync(S.L.graphs, S.hg.data(), sizeof(GraphArgs) * G, hipMemcpyHostToDevice, s));
    RWC_HIP(hipMemcpyAsync(S.L.node_off, S.plan.node_off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    RWC_HIP(hipMemcpyAsync(S.L.items, S.items.data(), sizeof(Item) * S.items.size(), hipMemcpyHostToDevice, s));
    return RWC_OK;
}

// ------------------------------------------------------------------------------------
// Workspaces prepared for a caller's stream capture: the device tables a call reads are a
// function of the graphs, the parameters (all but seed and sample_begin) and the workspace,
// summarised by a signature.  rwc_sample_prepare uploads them and records the signature; a
// call on a capturing stream checks it and launches kernels only (a capture cannot hold the
// host-to-device copies, whose source memory would not outlive the call).
// ------------------------------------------------------------------------------------
struct KeyBuilder {
    std::vector<uint64_t> words;
    template <class T>
    void add_bytes(const T& v) {
        uint64_t w[(sizeof(T) + 7) / 8] = {};
        std::memcpy(w, &v, sizeof(T));
        for (uint64_t x : w) words.push_back(x);
    }
    void add(uint64_t x) { words.push_back(x); }
};

std::vector<uint64_t> table_signature(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p, const void* ws,
                                      size_t ws_bytes) {
    KeyBuilder k;
    k.add(static_cast<uint64_t>(G));
    for (int32_t g = 0; g < G; ++g) k.add_bytes(graphs[g]);
    rwc_sample_params q = *p;
    q.seed = 0;
    q.sample_begin = 0;
    q.flags &= ~(RWC_SAMPLE_ACCUMULATE | RWC_SAMPLE_GRAPH_CAPTURE);
    q.walkers_per_graph = nullptr;   // the contents count, not where the host keeps them
    k.add_bytes(q);
    if (p->walkers_per_graph)
        for (int32_t g = 0; g < G; ++g) k.add(static_cast<uint64_t>(p->walkers_per_graph[g]));
    k.add(reinterpret_cast<uintptr_t>(ws));
    k.add(static_cast<uint64_t>(ws_bytes));
    return k.words;
}

std::mutex g_prep_mu;
std::unordered_map<const void*, std::vector<uint64_t>> g_prepared;

// ------------------------------------------------------------------------------------
// RWC_SAMPLE_GRAPH_CAPTURE: the launches of a call are captured once into a hipGraph and the
// instantiated graph is kept, keyed by everything its kernels take as arguments (the table
// signature, seed, sample range, flags, output pointers, parent dumps); a later call with the
// same key uploads the tables and replays it.  At most kExecCache graphs are kept.
// ------------------------------------------------------------------------------------
constexpr size_t kExecCache = 8;
struct CachedExec {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
    uint64_t used = 0;
};
std::mutex g_exec_mu;
std::vector<CachedExec> g_execs;
uint64_t g_exec_clock = 0;

void destroy_exec(CachedExec& e) {   // teardown: failures here have nobody to report to
    if (e.last_stream) (void)hipStreamSynchronize(e.last_stream);
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_sample_forests_workspace(const rwc_csr* graphs, int32_t num_graphs, const rwc_sample_params* p,
                                            size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(validate(graphs, num_graphs, p));
    Plan plan;
    RWC_CHECK(make_plan(graphs, num_graphs, p, &plan));
    *bytes = carve_sample(nullptr, num_graphs, plan, graphs[0].n, p->num_samples).total;
    return RWC_OK;
}

extern "C" int rwc_sample_prepare(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p, void* ws,
                                  size_t ws_bytes, void* stream) {
    clear_error();
    RWC_CHECK(validate(graphs, G, p));
    Setup S;
    {
        Plan plan;
        RWC_CHECK(make_plan(graphs, G, p, &plan));
        RWC_CHECK(check_workspace(ws, ws_bytes, carve_sample(nullptr, G, plan, graphs[0].n, p->num_samples).total));
    }
    RWC_CHECK(make_setup(graphs, G, p, ws, &S));
    hipStream_t s = static_cast<hipStream_t>(stream);
    RWC_CHECK(upload_tables(S, G, s));
    RWC_HIP(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> lock(g_prep_mu);
    g_prepared[ws] = table_signature(graphs, G, p, ws, ws_bytes);
    return RWC_OK;
}

extern "C" void rwc_release_cached_graphs(void) {
    std::lock_guard<std::mutex> lock(g_exec_mu);
    for (auto& e : g_execs) destroy_exec(e);
    g_execs.clear();
}

extern "C" int rwc_sample_forests(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p,
                                  const rwc_sample_outputs* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    RWC_CHECK(validate(graphs, G, p));
    if (!out || !out->counts) return fail(RWC_ERR_INVALID_ARG, "out->counts is required");
    if (out->ndump < 0 || out->ndump > kMaxDump) return fail(RWC_ERR_INVALID_ARG, "ndump must be in [0, %d]", kMaxDump);
    if (out->ndump > 0 && (G != 1 || !out->parents || !out->dump_samples))
        return fail(RWC_ERR_INVALID_ARG, "parent dumps need a single graph, parents and dump_samples");
    for (int d = 0; d < out->ndump; ++d)
        if (out->dump_samples[d] < p->sample_begin || out->dump_samples[d] >= p->sample_begin + p->num_samples)
            return fail(RWC_ERR_INVALID_ARG, "dump sample %lld is outside the sampled range",
                        (long long)out->dump_samples[d]);
    const bool capture = (p->flags & RWC_SAMPLE_GRAPH_CAPTURE) != 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    if (s != nullptr) RWC_HIP(hipStreamIsCapturing(s, &cst));   // the legacy default stream is never captured
    const bool caller_capture = (cst != hipStreamCaptureStatusNone);
    if ((capture || caller_capture) && out->timing_ms)
        return fail(RWC_ERR_INVALID_ARG, "timing_ms is not available in a captured call");
    if (capture && caller_capture)
        return fail(RWC_ERR_INVALID_ARG, "RWC_SAMPLE_GRAPH_CAPTURE on a stream that is being captured");
    {
        Plan plan;
        RWC_CHECK(make_plan(graphs, G, p, &plan));
        RWC_CHECK(check_workspace(ws, ws_bytes, carve_sample(nullptr, G, plan, graphs[0].n, p->num_samples).total));
    }
    if (caller_capture) {
        std::lock_guard<std::mutex> lock(g_prep_mu);
        auto it = g_prepared.find(ws);
        if (it == g_prepared.end() || it->second != table_signature(graphs, G, p, ws, ws_bytes))
            return fail(RWC_ERR_INVALID_ARG,
                        "a call on a capturing stream needs a workspace prepared by rwc_sample_prepare "
                        "with the same graphs and parameters");
    }
    Setup S;
    RWC_CHECK(make_setup(graphs, G, p, ws, &S));
    const Plan& plan = S.plan;
    const SampleLayout& L = S.L;
    const int64_t l = p->num_samples;
    const int32_t nit = S.nit_hbm;
    const bool persistent = (p->flags & RWC_SAMPLE_PERSISTENT) != 0;
    if (!caller_capture) RWC_CHECK(upload_tables(S, G, s));

    Timer timer;
    if (out->timing_ms) RWC_CHECK(timer.init());
    const int32_t nroots = p->num_roots;
    auto launches = [&](hipStream_t ls) -> int {
        const unsigned node_blocks = blocks_for(plan.total_nodes, 256) < 8192 ? blocks_for(plan.total_nodes, 256) : 8192;
        const bool accumulate = (p->flags & RWC_SAMPLE_ACCUMULATE) != 0;
        hipLaunchKernelGGL(zero_outputs, dim3(node_blocks), dim3(256), 0, ls, accumulate ? nullptr : out->counts,
                           accumulate ? nullptr : out->counts_sq, plan.total_nodes,
                           accumulate ? nullptr : out->total_steps, G, L.header, L.queue, L.rootmask,
                           nroots > 0 ? L.mask_words : int64_t{0});
        if (nroots > 0)
            hipLaunchKernelGGL(build_rootmask, dim3(blocks_for(nroots, 256)), dim3(256), 0, ls, p->roots, nroots,
                               graphs[0].n, graphs[0].node_index, L.rootmask, L.header);
        if (nroots > 0 && graphs[0].components > 1)
            check_root_cover(graphs[0], p->roots, nroots, L.cover, L.rootmask, L.header, ls);
        if (p->root >= 0) hipLaunchKernelGGL(resolve_root, dim3(1), dim3(1), 0, ls, L.graphs, graphs[0].node_index, p->root);
        hipLaunchKernelGGL(init_state, dim3(node_blocks), dim3(256), 0, ls, L.graphs, L.node_off, G, plan.total_nodes);
        for (int32_t b = 0; b < plan.batches; ++b) {
            // every graph runs its samples [b*T_g, (b+1)*T_g); graphs with fewer batches idle
            if (out->timing_ms) RWC_HIP(hipEventRecord(timer.ev[0], ls));
            uint32_t* status = &L.header->status;
            if (b == 0 && S.nit_lds > 0) {
                // every tree of the LDS-state graphs, in one persistent launch
                DumpArgs ldumps{};
                if (plan.lds[0])
                    for (int d = 0; d < out->ndump; ++d) {
                        ldumps.slot[ldumps.count] = static_cast<int32_t>(out->dump_samples[d] - p->sample_begin);
                        ldumps.out[ldumps.count] = d;
                        ++ldumps.count;
                    }
                hipLaunchKernelGGL(S.walk_lds, dim3(S.grid_lds), dim3(kWave), S.lds_bytes, ls, L.graphs,
                                   L.items + S.nit_hbm, S.nit_lds, L.queue + 1, p->sample_begin, l, p->seed, L.node_off,
                                   out->counts, out->counts_sq, out->parents, ldumps, out->tree_hash, out->total_steps,
                                   status);
            }
            if (nit > 0 && persistent) {
                hipLaunchKernelGGL(reset_queue, dim3(1), dim3(1), 0, ls, L.queue);
                const int grid = S.grid_persistent < nit ? S.grid_persistent : nit;
                hipLaunchKernelGGL(S.walk, dim3(grid), dim3(kWave), 0, ls, L.graphs, L.items, nit, L.queue, b,
                                   p->sample_begin, l, p->seed, out->tree_hash, out->total_steps, status);
            } else if (nit > 0) {
                hipLaunchKernelGGL(S.walk, dim3(nit), dim3(kWave), 0, ls, L.graphs, L.items, nit, nullptr, b,
                                   p->sample_begin, l, p->seed, out->tree_hash, out->total_steps, status);
            }
            DumpArgs dumps{};
            for (int d = 0; d < out->ndump && !plan.lds[0]; ++d) {
                const int64_t rel = out->dump_samples[d] - p->sample_begin - static_cast<int64_t>(b) * plan.T[0];
                if (rel >= 0 && rel < plan.T[0]) {
                    dumps.slot[dumps.count] = static_cast<int32_t>(rel);
                    dumps.out[dumps.count] = d;
                    ++dumps.count;
                }
            }
            if (out->timing_ms) RWC_HIP(hipEventRecord(timer.ev[1], ls));
            hipLaunchKernelGGL(reduce_batch, dim3(node_blocks), dim3(256), 0, ls, L.graphs, L.node_off, G,
                               plan.total_nodes, b, l, b + 1 < plan.batches, out->counts, out->counts_sq,
                               out->parents, dumps);
            if (out->timing_ms) {
                RWC_HIP(hipEventRecord(timer.ev[2], ls));
                RWC_HIP(hipEventSynchronize(timer.ev[2]));
                float a = 0.f, c = 0.f;
                RWC_HIP(hipEventElapsedTime(&a, timer.ev[0], timer.ev[1]));
                RWC_HIP(hipEventElapsedTime(&c, timer.ev[1], timer.ev[2]));
                timer.walk_ms += a;
                timer.reduce_ms += c;
            }
        }
        RWC_HIP(hipGetLastError());
        return RWC_OK;
    };

    int32_t replayed = -1;
    if (capture) {
        KeyBuilder k;
        k.words = table_signature(graphs, G, p, ws, ws_bytes);
        k.add(p->seed);
        k.add(static_cast<uint64_t>(p->sample_begin));
        k.add(p->flags);
        for (const void* q : {static_cast<const void*>(out->counts), static_cast<const void*>(out->counts_sq),
                              static_cast<const void*>(out->total_steps), static_cast<const void*>(out->tree_hash),
                              static_cast<const void*>(out->parents)})
            k.add(reinterpret_cast<uintptr_t>(q));
        k.add(static_cast<uint64_t>(out->ndump));
        for (int d = 0; d < out->ndump; ++d) k.add(static_cast<uint64_t>(out->dump_samples[d]));
        std::lock_guard<std::mutex> lock(g_exec_mu);
        CachedExec* hit = nullptr;
        for (auto& e : g_execs)
            if (e.key == k.words) hit = &e;
        const bool replay = hit != nullptr;
        if (!hit) {
            if (g_execs.size() >= kExecCache) {
                auto lru = std::min_element(g_execs.begin(), g_execs.end(),
                                            [](const CachedExec& a, const CachedExec& b) { return a.used < b.used; });
                destroy_exec(*lru);
                g_execs.erase(lru);
            }
            // capture on a private stream (the caller's may be the legacy default stream, which
            // cannot be captured); nothing runs during the capture
            hipStream_t cs = nullptr;
            RWC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            CachedExec e;
            e.key = k.words;
            int rc = RWC_OK;
            hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (he == hipSuccess) {
                rc = launches(cs);
                he = hipStreamEndCapture(cs, &e.graph);
            }
            (void)hipStreamDestroy(cs);
            if (rc == RWC_OK && he == hipSuccess) he = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
            if (rc != RWC_OK || he != hipSuccess) {
                destroy_exec(e);
                if (rc != RWC_OK) return rc;
                return fail(RWC_ERR_HIP, "hipGraph capture of the sampler failed: %s", hipGetErrorString(he));
            }
            g_execs.push_back(std::move(e));
            hit = &g_execs.back();
        }
        hit->used = ++g_exec_clock;
        hit->last_stream = s;
        RWC_HIP(hipGraphLaunch(hit->exec, s));
        replayed = replay ? 1 : 0;
    } else {
        RWC_CHECK(launches(s));
    }
    if (out->plan) {
        // graph 0's plan (every graph's plan is the same unless chosen automatically)
        out->plan[0] = plan.W[0];
        out->plan[1] = plan.T[0];
        out->plan[2] = plan.batches;
        out->plan[3] = plan.lds[0] ? (S.lds_ring ? 4 : 3) : (!plan.team ? 0 : (S.ring ? 2 : 1));
        out->plan[4] = S.hg[0].spread;
        out->plan[5] = S.hg[0].order != nullptr ? 1 : 0;
        out->plan[6] = replayed;
        out->plan[7] = plan.lds_graphs;
    }
    if (out->timing_ms) {
        out->timing_ms[0] = timer.walk_ms;
        out->timing_ms[1] = timer.reduce_ms;
        // the call has synchronised already: report the device status now
        WsHeader h{};
        RWC_HIP(hipMemcpyAsync(&h, L.header, sizeof(h), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
        return device_error_to_status(h.status);
    }
    return RWC_OK;
}
