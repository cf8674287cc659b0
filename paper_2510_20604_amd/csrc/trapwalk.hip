// rwc_sample_trap_walks: the trap-walk estimator of the diagonal of calL_v^{-1} (Lemma 5.1 and
// the method the paper describes after it, which FastWalk improves on): from every node u != v,
// l independent random walks that stop at the trap v, each counting its visits to u (the start
// included); the mean count estimates t_u = (calL_v^{-1})_uu, the same quantity the Wilson
// forests' visit totals estimate, so rwc_estimate assembles RWC from either.
//
// The walks keep no per-walk memory besides registers: a lane holds one walk (start u, walk
// index i, position x, step s, visit count) and each step reads only the record of x (and the
// row when the draw lands past the record), so the kernel is a pure chain of dependent
// gathers.  Walk i from u takes its s-th step with Philox4x32-10 on (s, u, i, graph ^ 2^31).
// Walks are numbered w = (i - walk_begin) (n - 1) + j with start node u = j (+1 past the trap),
// so neighbouring lanes start from different nodes; a wave hands the walks of finished lanes
// out again from a device counter (one atomic per refill), so lanes stay busy until the
// numbered walks run out.
#include "common.hpp"
#include "device.hpp"
#include "select.hpp"

namespace rwc {
namespace {

struct TrapArgs {
    const int32_t* col;
    const uint64_t* cdf;
    const uint4* rec;
    const int32_t* node_index;   // internal index of each input id
    uint64_t* counts;
    uint64_t* counts_sq;
    uint64_t* total_steps;
    uint32_t* queue;
    WsHeader* header;
    uint64_t total_walks;
    uint64_t max_steps;
    int64_t walk_begin;
    uint64_t seed;
    int32_t n;
    int32_t trap;                // input id
    uint32_t graph_word;
};

__global__ void trap_begin(WsHeader* header, uint32_t* queue, uint64_t* counts, uint64_t* counts_sq,
                           uint64_t* total_steps, int32_t n) {
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    for (int64_t i = tid; i < n; i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        counts[i] = 0;
        if (counts_sq) counts_sq[i] = 0;
    }
    if (tid == 0) {
        header_begin(header);
        queue[0] = 0;
        queue[1] = 0;
        if (total_steps) *total_steps = 0;
    }
}

__global__ void __launch_bounds__(kWave) trap_walks(TrapArgs A) {
    const int lane = threadIdx.x & (kWave - 1);
    const auto col = global_ptr(A.col);
    const auto cdf = global_ptr(A.cdf);
    const auto rec = global_ptr(A.rec);
    const uint32_t k0 = static_cast<uint32_t>(A.seed), k1 = static_cast<uint32_t>(A.seed >> 32);
    const uint64_t starts = static_cast<uint64_t>(A.n - 1);
    // the walk counter is 64 bits wide: two 32-bit words updated by one 64-bit atomic
    auto* q64 = reinterpret_cast<unsigned long long*>(A.queue);
    // walks are enumerated and keyed by input ids (u); the walk itself moves over internal
    // indices (x, y; xs the start's, trap_x the trap's)
    const uint32_t trap_x = static_cast<uint32_t>(A.node_index[A.trap]);
    bool busy = false, done = false;
    uint32_t u = 0, x = 0, xs = 0, count = 0;
    uint32_t i = 0;
    uint64_t s = 0, steps = 0;
    uint32_t err = 0;
    while (true) {
        // refill idle lanes
        const bool idle = !busy && !done;
        const uint64_t want = __ballot(idle);
        if (want) {
            unsigned long long base = 0;
            if (lane == __ffsll(static_cast<long long>(want)) - 1)
                base = atomicAdd(q64, static_cast<unsigned long long>(__popcll(want)));
            base = __shfl(base, __ffsll(static_cast<long long>(want)) - 1, kWave);
            if (idle) {
                const uint64_t w = base + __popcll(want & ((1ull << lane) - 1ull));
                if (w < A.total_walks) {
                    const uint64_t j = w % starts;
                    i = static_cast<uint32_t>(static_cast<uint64_t>(A.walk_begin) + w / starts);
                    u = static_cast<uint32_t>(j) + (static_cast<int64_t>(j) >= A.trap ? 1u : 0u);
                    xs = static_cast<uint32_t>(A.node_index[u]);
                    x = xs;
                    s = 0;
                    count = 1;
                    busy = true;
                } else {
                    done = true;
                }
            }
        }
        if (__all(done)) break;
        if (busy) {
            const auto q = rec + (kRecWords / 4) * static_cast<int64_t>(x);
            const uint4 ra = load_u4(q + 0), rb = load_u4(q + 1), rc = load_u4(q + 2), rd = load_u4(q + 3);
            const uint64_t r = philox_x64(static_cast<uint32_t>(s), u, i, A.graph_word, k0, k1);
            const uint32_t y = choose_neighbor(r, [&](uint32_t t) { return rec_word(ra, rb, rc, rd, t); }, col, cdf);
            ++s;
            if (y == trap_x) {
                atomicAdd(reinterpret_cast<unsigned long long*>(&A.counts[u]), static_cast<unsigned long long>(count));
                if (A.counts_sq)
                    atomicAdd(reinterpret_cast<unsigned long long*>(&A.counts_sq[u]),
                              static_cast<unsigned long long>(count) * count);
                steps += s;
                busy = false;
            } else if (s >= A.max_steps) {
                err |= kErrStepLimit;
                steps += s;
                busy = false;
            } else {
                count += (y == xs) ? 1u : 0u;
                x = y;
            }
        }
    }
    const uint64_t ws = wave_sum(steps);
    if (lane == 0 && A.total_steps && ws)
        atomicAdd(reinterpret_cast<unsigned long long*>(A.total_steps), static_cast<unsigned long long>(ws));
    if (err) atomicOr(&A.header->status, err);
}

struct TrapLayout {
    WsHeader* header;
    uint32_t* queue;
    size_t total;
};

TrapLayout carve_trap(void* ws) {
    Carver c(ws);
    TrapLayout L{};
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.queue = c.take<uint32_t>(2);
    L.total = c.used();
    return L;
}

int check_trap(const rwc_csr* g, const rwc_trap_params* p) {
    if (!g || !p) return fail(RWC_ERR_INVALID_ARG, "g and p are required");
    if (g->n < 2 || !g->rec || !g->col) return fail(RWC_ERR_INVALID_ARG, "g is not a built CSR");
    if (p->num_walks < 1 || p->walk_begin < 0 || p->num_walks > (int64_t{1} << 32) ||
        p->walk_begin > (int64_t{1} << 32) - p->num_walks)
        return fail(RWC_ERR_INVALID_ARG, "walk indices must lie in [0, 2^32)");
    if (p->trap >= g->n) return fail(RWC_ERR_INVALID_ARG, "trap out of range");
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_sample_trap_walks_workspace(const rwc_csr* g, const rwc_trap_params* p, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(check_trap(g, p));
    *bytes = carve_trap(nullptr).total;
    return RWC_OK;
}

extern "C" int rwc_sample_trap_walks(const rwc_csr* g, const rwc_trap_params* p, uint64_t* counts,
                                     uint64_t* counts_sq, uint64_t* total_steps, void* ws, size_t ws_bytes,
                                     void* stream) {
    clear_error();
    RWC_CHECK(check_trap(g, p));
    RWC_CHECK(require_connected(g, "rwc_sample_trap_walks"));
    if (!counts) return fail(RWC_ERR_INVALID_ARG, "counts is required");
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_trap(nullptr).total));
    TrapLayout L = carve_trap(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    TrapArgs A{};
    A.col = g->col;
    A.cdf = g->weighted ? g->cdf : nullptr;
    A.rec = reinterpret_cast<const uint4*>(g->rec);
    A.node_index = g->node_index;
    A.counts = counts;
    A.counts_sq = counts_sq;
    A.total_steps = total_steps;
    A.queue = L.queue;
    A.header = L.header;
    A.total_walks = static_cast<uint64_t>(g->n - 1) * static_cast<uint64_t>(p->num_walks);
    A.max_steps = p->max_steps_per_walk ? p->max_steps_per_walk : (1ull << 20) + 4096ull * static_cast<uint64_t>(g->n);
    A.walk_begin = p->walk_begin;
    A.seed = p->seed;
    A.n = g->n;
    A.trap = p->trap >= 0 ? p->trap : g->pivot;
    A.graph_word = p->graph_index ^ 0x80000000u;
    hipLaunchKernelGGL(trap_begin, dim3(blocks_for(g->n, 256) < 4096 ? blocks_for(g->n, 256) : 4096), dim3(256), 0, s,
                       L.header, L.queue, counts, counts_sq, total_steps, g->n);
    // persistent grid: every resident wave slot, capped by the walks
    static int per_cu = 0;
    if (per_cu == 0) {
        RWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trap_walks, kWave, 0));
        if (per_cu < 1) per_cu = 1;
    }
    int64_t grid = static_cast<int64_t>(per_cu) * device_cu_count();
    const int64_t need = static_cast<int64_t>((A.total_walks + kWave - 1) / kWave);
    if (grid > need) grid = need;
    hipLaunchKernelGGL(trap_walks, dim3(static_cast<unsigned>(grid)), dim3(kWave), 0, s, A);
    RWC_HIP(hipGetLastError());
    return RWC_OK;
}
