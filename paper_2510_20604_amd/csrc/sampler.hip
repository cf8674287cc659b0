// rwc_sample_forests: Wilson's algorithm (Section 5, Algorithm 3) on the GPU, many trees at
// once, with the visit counting of Algorithm 3 reduced into per-node totals.
//
// Layout.  Each graph g keeps T tree slots; slot t holds one 64-bit state word per node
// (state[t * n_g + u], see device.hpp) -- the InTree flag, Next[u] and the departure count
// of u in the slot's current tree.  A batch runs T trees (one per slot) to completion, then a
// reduction pass folds the per-tree departure counts into the per-node totals, writes the
// requested parent dumps and resets the slots for the next batch.
//
// Two kernels.  wilson_walk: one lane grows one tree, running Algorithm 3's three loops --
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
#include <numeric>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace rwc {
namespace {

struct GraphArgs {
    const int32_t* row_ptr;
    const int32_t* col;
    const uint64_t* cdf;
    const uint4* rec;       // 64-byte node records (4 x uint4 per node)
    const int32_t* order;   // start order of walker teams (breadth-first from the pivot)
    uint64_t* state;        // [T][stride]
    int64_t stride;         // words per tree slot (n rounded up to a multiple of 8)
    uint64_t guard;         // per-tree step guard (one walker) or iteration guard (team)
    int32_t n;
    int32_t root;
    uint32_t graph_word;
    int32_t T;              // tree slots (trees in flight) of this graph
    int32_t W;              // walkers per tree
    int32_t spread;         // each walker of a team takes starts from its own range
};

struct Item {
    int32_t graph;
    int32_t slot0;
};

constexpr int kMaxDump = 64;

struct DumpArgs {
    int32_t count;
    int32_t slot[kMaxDump];
    int32_t out[kMaxDump];
};

enum Phase : int { kScan = 0, kWalk = 1, kRetrace = 2, kDone = 3 };

// Word i (0..15) of a node record held in four uint4 registers.
__device__ __forceinline__ uint32_t rec_word(const uint4& a, const uint4& b, const uint4& c, const uint4& d,
                                             uint32_t i) {
    const uint4 q = (i < 4) ? a : (i < 8) ? b : (i < 12) ? c : d;
    const uint32_t s = i & 3u;
    return s == 0 ? q.x : (s == 1 ? q.y : (s == 2 ? q.z : q.w));
}

// RandomNeighbor (Algorithm 3): the neighbour id chosen at a node by the 64 random bits x,
// read from the node's record wherever it holds the answer.  rec(i) returns word i of the
// record, already local (registers or LDS).  Unweighted: position floor(x deg / 2^64), inline
// below kRecInline.  Weighted: the first position k with floor(x S / 2^64) < cdf[k], S the
// row's total; the record's four CDF values settle it without a read of the row whenever r
// falls below the fourth, else a binary search over the rest of the row's CDF does.
template <class Rec>
__device__ __forceinline__ uint32_t choose_neighbor(uint64_t x, Rec rec, const RWC_GLOBAL int32_t* col,
                                                    const RWC_GLOBAL uint64_t* cdf) {
    const uint32_t deg = rec(0);
    const int32_t beg = static_cast<int32_t>(rec(1));
    uint32_t pos;
    if (cdf == nullptr) {
        pos = static_cast<uint32_t>(select_unweighted(x, static_cast<int32_t>(deg)));
        if (pos < static_cast<uint32_t>(kRecInline)) return rec(2u + pos);
    } else {
        const uint64_t total = rec(6) | (static_cast<uint64_t>(rec(7)) << 32);
        const uint64_t r = mulhi64(x, total);
        uint64_t c[kRecInlineWeighted];
#pragma unroll
        for (int i = 0; i < kRecInlineWeighted; ++i)
            c[i] = rec(8u + 2u * i) | (static_cast<uint64_t>(rec(9u + 2u * i)) << 32);
        if (deg <= static_cast<uint32_t>(kRecInlineWeighted) || r < c[kRecInlineWeighted - 1]) {
            // the CDF is non-decreasing and exceeds r at position lim, so the first position
            // above r is the number of positions below lim whose value is <= r
            const uint32_t lim = (deg < static_cast<uint32_t>(kRecInlineWeighted) ? deg : kRecInlineWeighted) - 1u;
            pos = 0;
#pragma unroll
            for (int i = 0; i < kRecInlineWeighted - 1; ++i)
                pos += (static_cast<uint32_t>(i) < lim && c[i] <= r) ? 1u : 0u;
            return rec(2u + pos);
        }
        int32_t lo = kRecInlineWeighted, hi = static_cast<int32_t>(deg) - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (r < cdf[beg + mid])
                hi = mid;
            else
                lo = mid + 1;
        }
        pos = static_cast<uint32_t>(lo);
    }
    return static_cast<uint32_t>(col[beg + static_cast<int32_t>(pos)]);
}

// Grows the tree of slot `slot` for absolute sample `sample` (one lane).
__device__ __forceinline__ void grow_tree(const GraphArgs& G, int32_t slot, uint64_t sample, uint64_t seed,
                                          bool want_hash, uint64_t& steps_out, uint64_t& hash_out,
                                          uint32_t& err_out) {
    const uint64_t max_steps = G.guard;
    const int32_t n = G.n;
    const auto row_ptr = global_ptr(G.row_ptr);
    const auto col = global_ptr(G.col);
    const auto cdf = global_ptr(G.cdf);
    const auto rec = global_ptr(G.rec);
    const auto st = global_ptr(G.state + static_cast<int64_t>(slot) * G.stride);
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const uint32_t sw = static_cast<uint32_t>(sample);
    const uint32_t gw = G.graph_word;
    // record of node rh_node, loaded with that node's state word when the walk arrives
    uint4 ra = make_uint4(0, 0, 0, 0), rb = ra, rc = ra, rd = ra;
    uint32_t rh_node = 0xFFFFFFFFu;

    uint32_t j = 0;      // next start candidate (ascending order, Algorithm 3)
    uint32_t x = 0;      // walk position, or retrace cursor
    uint32_t hit = 0;    // node at which the current walk met the tree
    uint64_t wx = 0;     // state word of x while walking
    uint64_t steps = 0, h = 0;
    uint32_t retr = 0, err = 0;
    int phase = kScan;
    while (phase != kDone) {
        if (phase == kScan) {
            if (j >= static_cast<uint32_t>(n)) {
                phase = kDone;
            } else {
                const uint64_t w = st[j];
                if (w & kInTree) {
                    ++j;
                } else {
                    x = j;
                    wx = w;
                    phase = kWalk;
                }
            }
        } else if (phase == kWalk) {
            const uint32_t k = st_cnt(wx);
            if (rh_node != x) {
                const auto q = rec + (kRecWords / 4) * static_cast<int64_t>(x);
                ra = load_u4(q + 0);
                rb = load_u4(q + 1);
                rc = load_u4(q + 2);
                rd = load_u4(q + 3);
                rh_node = x;
            }
            const uint64_t r = philox_x64(k, x, sw, gw, k0, k1);
            const uint32_t y = choose_neighbor(r, [&](uint32_t i) { return rec_word(ra, rb, rc, rd, i); }, col, cdf);
            st[x] = st_make(y, k + 1);
            const uint64_t wy = st[y];
            {
                const auto q = rec + (kRecWords / 4) * static_cast<int64_t>(y);   // y is the next position
                ra = load_u4(q + 0);
                rb = load_u4(q + 1);
                rc = load_u4(q + 2);
                rd = load_u4(q + 3);
                rh_node = y;
            }
            ++steps;
            if (k + 1 >= kCntMax) {
                err |= kErrCountOverflow;
                phase = kDone;
            } else if (steps > max_steps) {
                err |= kErrStepLimit;
                phase = kDone;
            } else if (wy & kInTree) {
                hit = y;
                x = j;
                retr = 0;
                phase = kRetrace;
            } else {
                x = y;
                wx = wy;
            }
        } else {  // kRetrace: mark the loop-erased path j -> ... -> hit
            if (x == hit) {
                ++j;
                phase = kScan;
            } else {
                const uint64_t w = st[x];
                const uint32_t p = st_next(w);
                st[x] = w | kInTree;
                if (want_hash) h += splitmix64((static_cast<uint64_t>(x) << 32) | p);
                x = p;
                if (++retr > static_cast<uint32_t>(n)) {
                    err |= kErrRetrace;
                    phase = kDone;
                }
            }
        }
    }
    steps_out = steps;
    hash_out = h;
    err_out = err;
}

// Batch b of graph g covers samples sample_begin + b*T_g + slot for slot in [0, T_g).
__device__ __forceinline__ void run_item(const GraphArgs* __restrict__ graphs, const Item it, int32_t batch,
                                         int64_t sample_begin, int64_t l, uint64_t seed,
                                         uint64_t* __restrict__ tree_hash, uint64_t* __restrict__ total_steps,
                                         uint32_t* __restrict__ status) {
    const int lane = threadIdx.x & (kWave - 1);
    const GraphArgs G = graphs[it.graph];
    const int32_t slot = it.slot0 + lane;
    const int64_t rel = static_cast<int64_t>(batch) * G.T + slot;   // sample index within the call
    uint64_t steps = 0, h = 0;
    uint32_t err = 0;
    const bool active = slot < G.T && rel < l;
    if (active) grow_tree(G, slot, static_cast<uint64_t>(sample_begin + rel), seed, tree_hash != nullptr, steps, h, err);
    if (active) {
        if (tree_hash) tree_hash[static_cast<int64_t>(it.graph) * l + rel] = h;
        if (err) atomicOr(status, err);
    }
    const uint64_t wsteps = wave_sum(steps);
    if (lane == 0 && total_steps && wsteps)
        atomicAdd(reinterpret_cast<unsigned long long*>(&total_steps[it.graph]),
                  static_cast<unsigned long long>(wsteps));
}

// One wave per work item (a block of 64 tree slots of one graph).  Persistent mode: a grid
// sized to the resident capacity pops items from `queue` until the list is exhausted.
__global__ void __launch_bounds__(kWave) wilson_walk(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                                     int32_t nitems, uint32_t* queue, int32_t batch,
                                                     int64_t sample_begin, int64_t l, uint64_t seed,
                                                     uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    if (queue == nullptr) {
        if (static_cast<int32_t>(blockIdx.x) < nitems)
            run_item(graphs, items[blockIdx.x], batch, sample_begin, l, seed, tree_hash, total_steps, status);
        return;
    }
    while (true) {
        uint32_t idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(queue, 1u);
        idx = __shfl(idx, 0, kWave);
        if (idx >= static_cast<uint32_t>(nitems)) break;
        run_item(graphs, items[idx], batch, sample_begin, l, seed, tree_hash, total_steps, status);
    }
}

// ---------------------------------------------------------------------------------------
// Several walkers per tree (a team of W lanes of one wave grows one tree).
//
// Wilson's algorithm is cycle popping on per-node stacks of random arrows: with the stack-keyed
// generator, any procedure that reads arrows in stack order and pops only genuine cycles of
// the current arrow configuration ends with the same tree and the same per-node departure
// counts as Algorithm 3's serial order.  A team runs W such walks at once:
//  * a walker owns the nodes of its current (loop-erased) path: state word OWNED + its team
//    lane id; its head's arrow is read at each step (departure count incremented);
//  * arrow into the tree       -> the path attaches (its nodes are marked INTREE: the newest
//                                 ones from the LDS ring at once, older ones by a chase from
//                                 the path's start).  The ring holds each buffered node with
//                                 its departure count, so its final word is written without
//                                 reading the old one;
//  * arrow into its own path   -> a cycle of its own arrows: the segment after the hit node is
//                                 released (FREE, counts kept) and the hit node is the head;
//  * arrow into a free node    -> claim it (compare-and-swap; the loser waits on the winner);
//  * arrow into another walker's path -> wait.  Waiting walkers whose targets form a cycle of
//    walkers hold a genuine arrow cycle: it is popped by every member releasing the segment
//    after its junction (the node its cycle predecessor points at), which becomes its head.
// Start nodes are handed out shared (a team takes consecutive positions of the start order)
// or spread (each walker its own contiguous range); a start owned by another walker is waited
// on until it is in the tree (skip) or free (claim).  Every iteration reads before it writes
// and ends with a work-group fence, so all lanes see one consistent snapshot per iteration.
// ---------------------------------------------------------------------------------------
constexpr uint32_t kPathBuf = 8;    // newest path nodes kept per walker (power of two)
// Weighted graphs whose mean degree (entries per node) exceeds this run without the path ring
// when they fill the device (see the plan).
constexpr int64_t kRingMaxMeanDegree = 16;
// Waiting walkers re-read their target, and the team looks for wait cycles, every kPollEvery-th
// iteration (a power of two): polls are reads that rarely change anything, and fewer of them
// leave the memory system to the walking lanes (256 mixed graphs: 7 % faster than every
// other iteration).
constexpr uint32_t kPollEvery = 8;

enum TeamMode : int { tIdle = 0, tStart = 1, tWalk = 2, tWait = 3, tRetrace = 4, tRelease = 5, tDone = 6 };

__device__ __forceinline__ uint64_t st_load(const RWC_GLOBAL uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_store(RWC_GLOBAL uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool st_cas(RWC_GLOBAL uint64_t* p, uint64_t expected, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool kRing>
__device__ void grow_team(const GraphArgs& G, int32_t slot, uint64_t sample, bool active, uint64_t seed,
                          uint2 (*lds_path)[kWave], uint4 (*lds_rec)[kWave],
                          bool want_hash, uint64_t& steps_out, uint64_t& hash_out, uint32_t& err_out) {
    constexpr uint32_t kNone = 64;
    constexpr uint32_t kNoNode = 0xFFFFFFFFu;
    const int W = G.W;                       // walkers per tree, a power of two <= 64
    const uint64_t max_iters = G.guard;
    const int lane = threadIdx.x & (kWave - 1);
    const int team = lane / W;
    const uint32_t tl = static_cast<uint32_t>(lane & (W - 1));
    const uint32_t team_base = static_cast<uint32_t>(team * W);
    const uint32_t n = static_cast<uint32_t>(G.n);
    const auto col = global_ptr(G.col);
    const auto cdf = global_ptr(G.cdf);
    const auto rec = global_ptr(G.rec);
    const auto order = global_ptr(G.order);
    const auto st = global_ptr(G.state + static_cast<int64_t>(slot) * G.stride);
    // record of node rh_node, loaded alongside that node's state word so that a step from a
    // fresh head needs no dependent load for low-degree rows.  It is copied straight from
    // memory into LDS (lane's column of lds_rec) without passing through registers; reads of
    // it wait for the copy with wait_vm().
    uint32_t rh_node = kNoNode;
    auto keep_record = [&](uint32_t v) {
        const auto q = rec + (kRecWords / 4) * static_cast<int64_t>(v);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_amdgcn_global_load_lds((const RWC_GLOBAL void*)(q + i),
                                             (RWC_LDS void*)(&lds_rec[i][0]), 16, 0, 0);
        rh_node = v;
    };
    auto rec_at = [&](uint32_t i) -> uint32_t {
        return reinterpret_cast<const uint32_t*>(&lds_rec[i >> 2][lane])[i & 3u];
    };
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const uint32_t sw = static_cast<uint32_t>(sample), gw = G.graph_word;

    uint32_t next_start = 0;                 // uniform within the team
    // spread starts: walker tl owns the start positions [tl*chunk, (tl+1)*chunk) of the order
    const uint32_t chunk = (n + static_cast<uint32_t>(W) - 1) / static_cast<uint32_t>(W);
    uint32_t my_next = tl * chunk;
    int mode = active ? tIdle : tDone;
    uint32_t j = 0;       // start of the current path
    uint32_t h = 0;       // head of the current path
    uint32_t hk = 0;      // departures from the head so far (its next arrow's index)
    uint32_t c = 0;       // node waited on (tWait) or chase cursor (tRetrace, tRelease)
    uint32_t cstop = 0;   // retrace (and release with the ring): stop once the next node is
                          // cstop; release without the ring: stop after cstop
    uint32_t jn = 0, jk = 0;   // release: the node that becomes the head afterwards, its count
    // ring of the newest nodes of this walker's path in LDS: entry 0 is the head and the
    // entries form a contiguous suffix of the path ending at it (nbuf >= 1 while walking).
    // An entry is (node, its departure count so far).  The departures of ring nodes live only
    // here: their state words keep the claim's (OWNED, owner, stale next and count), which
    // is all other walkers look at, and get their real word when they leave the ring (the
    // oldest entry, when a push finds the ring full) or their final word on attach or loop
    // erasure.  Chases therefore only ever walk nodes older than the ring.
    uint32_t nbuf = 0, bhead = 0;
    auto buf = [&](uint32_t d) -> uint32_t { return lds_path[(bhead - d) & (kPathBuf - 1)][lane].x; };
    auto buf_cnt = [&](uint32_t d) -> uint32_t { return lds_path[(bhead - d) & (kPathBuf - 1)][lane].y; };
    auto push = [&](uint32_t v, uint32_t cnt) {
        if constexpr (kRing) {
            if (nbuf == kPathBuf) {
                // the oldest entry leaves: its arrow points at the next-older entry's node
                const uint2 e = lds_path[(bhead + 1) & (kPathBuf - 1)][lane];
                const uint32_t next = lds_path[(bhead + 2) & (kPathBuf - 1)][lane].x;
                st_store(&st[e.x], st_make_owned(next, e.y, tl));
            }
            bhead = (bhead + 1) & (kPathBuf - 1);
            lds_path[bhead][lane] = make_uint2(v, cnt);
            nbuf = nbuf < kPathBuf ? nbuf + 1 : kPathBuf;
        }
    };
    auto find = [&](uint32_t v) -> uint32_t {   // offset of v among entries 1..nbuf-1, 0 if absent
        if constexpr (kRing) {
            for (uint32_t d = 1; d < nbuf; ++d)
                if (buf(d) == v) return d;
        }
        return 0u;
    };
    uint64_t steps = 0, hsum = 0, iters = 0;
    uint32_t err = 0;
    while (true) {
        // ---- hand out start nodes to idle walkers of each team
        const bool idle = (mode == tIdle);
        const uint64_t bi = __ballot(idle);
        // idle walkers of my team (bit t = team lane t)
        const uint64_t tbits = (W == kWave) ? bi : ((bi >> team_base) & ((1ull << W) - 1ull));
        if (idle) {
            // starts in ascending order, or breadth-first from the root on request; shared
            // (the team takes consecutive positions) or spread (each walker its own range).
            // Any order gives the same forest; it only changes how walks overlap in time.
            uint32_t idx;
            if (G.spread) {
                const uint32_t my_end = (tl + 1) * chunk < n ? (tl + 1) * chunk : n;
                idx = my_next < my_end ? my_next++ : n;
            } else {
                idx = next_start + static_cast<uint32_t>(__popcll(tbits & ((1ull << tl) - 1ull)));
            }
            mode = (idx < n) ? tStart : tDone;
            if (idx < n) j = order ? static_cast<uint32_t>(order[idx]) : idx;
        }
        next_start += static_cast<uint32_t>(__popcll(tbits));
        if (__all(mode == tDone)) break;
        if (++iters > max_iters) {
            err |= kErrStepLimit;
            break;
        }

        // ---- reads: the node this walker looks at in this iteration and its state word
        // (one load for all lanes, issued after the walk's neighbour choice)
        uint32_t node = 0;
        uint32_t k = 0;
        if (mode == tWalk) {
            if (rh_node != h) keep_record(h);
            wait_vm();
            k = hk;
            const uint64_t r = philox_x64(k, h, sw, gw, k0, k1);
            node = choose_neighbor(r, rec_at, col, cdf);
        } else if (mode == tStart) {
            node = j;
        } else if (mode == tWait || mode == tRetrace || mode == tRelease) {
            node = c;
        }
        // a waiting walker re-reads its target every kPollEvery-th iteration, the iterations
        // of the cycle checks, so those always see fresh words
        const bool reads =
            (mode != tDone) && (mode != tIdle) && (mode != tWait || (iters & (kPollEvery - 1u)) == 0);
        const uint64_t w = reads ? st_load(&st[node]) : 0ull;
        // A node's record (for the walk steps from it) is fetched once the node is known to
        // become the head -- a claim or a loop pop below -- not with every state read: most
        // walk steps end in the tree or on an owned node, most start checks find the node in
        // the tree and most polls find it still owned.  The copy lands while the rest of the
        // iteration runs; on BA(10^6) the saved traffic outweighs the later arrival by 19%.
        const bool w_tree = (w & kInTree) != 0;
        const bool w_owned = (w & kOwned) != 0;
        const bool w_mine = w_owned && st_owner(w) == tl;

        // ---- decide.  Writes of this iteration: without the ring, the departure word of the
        // head, issued as soon as it is known (no lane reads state words again before the
        // iteration's fence, and issuing it early lets it drain while the rest of the iteration
        // runs; measured faster than issuing it with the other writes), or one chase store;
        // then either a batch of final-word stores of ring entries or one compare-and-swap
        // claim of `node` (whose push may store the word of the entry leaving the ring).
        bool departed = false;
        uint32_t st_node = kNoNode;
        uint64_t st_word = 0;
        bool claim = false, waiting = false;
        constexpr int kActNone = 0, kActAttach = 1, kActPop = 2;
        int act = kActNone;
        uint32_t act_v = 0, act_k = 0, act_next = 0;   // attach: tree node hit; pop: kept node
        if (mode == tWalk) {
            // departure from the head along arrow k (with the ring: recorded in the head's
            // entry only)
            if constexpr (kRing)
                lds_path[bhead][lane].y = k + 1;
            else
                st_store(&st[h], st_make_owned(node, k + 1, tl));
            departed = true;
            ++steps;
            if (k + 1 >= kCntMax) {
                err |= kErrCountOverflow;
                mode = tDone;
            } else if (w_tree) {
                act = kActAttach;
                act_v = node;
            } else if (w_mine) {
                // own cycle node -> ... -> h -> node: keep node as the head, release the rest
                keep_record(node);
                act = kActPop;
                act_v = node;
                act_k = st_cnt(w);
                act_next = st_next(w);
            } else if (w_owned) {
                mode = tWait;
                c = node;
                waiting = true;
            } else {
                keep_record(node);
                claim = true;
            }
        } else if (mode == tStart) {
            if (w_tree)
                mode = tIdle;
            else if (!w_owned)
                claim = true;
        } else if (mode == tWait && !reads) {
            // nothing read this iteration
        } else if (mode == tWait) {
            if (w_tree) {
                act = kActAttach;
                act_v = c;
            } else if (!w_owned) {
                claim = true;
            } else if (w_mine) {
                err |= kErrProtocol;
                mode = tDone;
            } else {
                waiting = true;
            }
        } else if (mode == tRetrace || mode == tRelease) {
            if (!w_mine) {
                err |= kErrProtocol;
                mode = tDone;
            } else if (mode == tRetrace) {
                // chase of the path prefix older than the ring: mark it INTREE
                st_node = c;
                st_word = (w & ~(kOwned | (0x3Full << 56))) | kInTree;
                if (want_hash) hsum += splitmix64((static_cast<uint64_t>(c) << 32) | st_next(w));
                if (st_next(w) == cstop)
                    mode = tIdle;
                else
                    c = st_next(w);
            } else {
                // chase release of a popped segment: FREE, departure count kept
                st_node = c;
                st_word = st_make(0u, st_cnt(w));
                if (kRing ? st_next(w) == cstop : c == cstop) {
                    mode = tWalk;
                    h = jn;
                    hk = jk;
                    push(jn, jk);
                } else {
                    c = st_next(w);
                }
            }
        }

        // ---- pop cycles of waiting walkers (team-local functional graph, pointer doubling:
        // after 64 applications every chain has either left the waiting set or entered a
        // cycle, so the image of the 64-fold map is exactly the set of cycle members).  A
        // cycle stays until it is popped, so looking every kPollEvery-th iteration only delays
        // pops.
        if ((iters & (kPollEvery - 1u)) == 0 && __any(waiting)) {
            const uint32_t wf = waiting ? team_base + (st_owner(w) & (W - 1)) : kNone;
            uint32_t p = wf;
#pragma unroll
            for (int it = 0; it < 6; ++it) {
                const uint32_t q = __shfl(p, static_cast<int>(p & (kWave - 1)), kWave);
                p = (p == kNone) ? kNone : q;
            }
            uint64_t img = (p == kNone) ? 0ull : (1ull << p);
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) img |= __shfl_xor(img, off, kWave);
            const bool on_cycle = waiting && ((img >> lane) & 1ull);
            // each cycle member has exactly one predecessor on its cycle: a forward permute
            // (ds_permute: lane i's value lands in lane addr_i / 4, no LDS allocated) hands
            // every member the lane id of its predecessor; other lanes send to themselves
            const uint32_t dst = on_cycle ? wf : static_cast<uint32_t>(lane);
            const uint32_t got = static_cast<uint32_t>(__builtin_amdgcn_ds_permute(static_cast<int>(dst << 2), lane));
            const uint32_t pred = on_cycle ? got : static_cast<uint32_t>(lane);
            const uint32_t py = __shfl(c, static_cast<int>(pred), kWave);
            const uint64_t pw = __shfl(w, static_cast<int>(pred), kWave);
            if (on_cycle) {
                // the cycle enters my path at py: the arrows from py on are popped
                if (py == h) {
                    // only my head's arrow is popped; if I departed in this iteration the
                    // snapshot the predecessor read predates my departure
                    mode = tWalk;
                    if constexpr (kRing)
                        hk = buf_cnt(0);
                    else
                        hk = departed ? k + 1 : st_cnt(pw);
                } else {
                    act = kActPop;
                    act_v = py;
                    act_k = st_cnt(pw);
                    act_next = st_next(pw);
                }
            }
        }

        // ---- the two path actions
        uint32_t ring_cnt = 0, ring_head = 0;   // final words for the ring_cnt newest ring entries:
        bool ring_attach = false;               // INTREE (attach) or FREE (release)
        bool repush = false;                    // after the ring's release: jn becomes the head
        if (act == kActAttach) {
            // the path attaches at tree node act_v: the buffered suffix becomes INTREE now,
            // an older prefix is chased from the start afterwards
            mode = tRetrace;
            c = j;
            cstop = act_v;   // without a ring: the chase runs up to the head
            if (kRing && nbuf > 0) {
                ring_cnt = nbuf;
                ring_head = bhead;
                ring_attach = true;
                if (want_hash)
                    for (uint32_t d = 0; d < nbuf; ++d)
                        hsum += splitmix64((static_cast<uint64_t>(buf(d)) << 32) | (d == 0 ? act_v : buf(d - 1)));
                cstop = buf(nbuf - 1);
                if (cstop == j) mode = tIdle;
            }
        } else if (act == kActPop) {
            // keep act_v (on the path, older than the head) as the head and release what is
            // newer: from the ring if act_v is buffered, else the whole ring now and the older
            // part by a chase from act_v's successor
            const uint32_t d = find(act_v);
            mode = tWalk;
            if (d > 0) {
                ring_cnt = d;
                ring_head = bhead;
                bhead = (bhead - d) & (kPathBuf - 1);
                nbuf -= d;
                h = act_v;
                if constexpr (kRing)
                    hk = buf_cnt(0);   // the ring holds act_v's current count
                else
                    hk = act_k;
            } else if constexpr (kRing) {
                ring_cnt = nbuf;
                ring_head = bhead;
                jn = act_v;
                jk = act_k;
                cstop = buf(nbuf - 1);
                if (act_next == cstop) {
                    repush = true;   // nothing older to release
                } else {
                    mode = tRelease;
                    c = act_next;
                }
                nbuf = 0;
            } else {
                mode = tRelease;
                c = act_next;
                cstop = h;
                jn = act_v;
                jk = act_k;
                nbuf = 0;
            }
        }

        // ---- writes (a lane that writes ring entries does not claim in the same iteration).
        // Ring entries carry their departure counts, so their final words are plain stores
        // (only the owner writes an owned node's word): no read of the old word, no fetch of
        // its line.
        if (st_node != kNoNode) st_store(&st[st_node], st_word);
        if constexpr (kRing) {
            uint32_t next = act_v;   // the newest entry's arrow points at the tree node hit
            for (uint32_t d = 0; d < ring_cnt; ++d) {
                const uint2 e = lds_path[(ring_head - d) & (kPathBuf - 1)][lane];
                st_store(&st[e.x], ring_attach ? (kInTree | st_make(next, e.y)) : st_make(0u, e.y));
                next = e.x;
            }
            if (repush) {
                mode = tWalk;
                h = jn;
                hk = jk;
                push(jn, jk);
            }
        }
        // keep the chase store ahead of the claim, so that both are in flight together
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (claim) {
            if (mode != tWalk) keep_record(node);
            const uint64_t want = st_make_owned(st_next(w), st_cnt(w), tl);
            if (st_cas(&st[node], w, want)) {
                if (mode == tStart) nbuf = 0;   // a start claim begins a new path at j
                h = node;
                hk = st_cnt(w);
                mode = tWalk;
                push(node, hk);
            } else if (mode == tWalk) {
                mode = tWait;     // lost the race: the winner owns the node now
                c = node;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    steps_out = steps;
    hash_out = hsum;
    err_out = err;
}

template <bool kRing>
__device__ __forceinline__ void run_team_item(const GraphArgs* __restrict__ graphs, const Item it, int32_t batch,
                                              int64_t sample_begin, int64_t l, uint64_t seed,
                                              uint2 (*lds_path)[kWave], uint4 (*lds_rec)[kWave],
                                              uint64_t* __restrict__ tree_hash, uint64_t* __restrict__ total_steps,
                                              uint32_t* __restrict__ status) {
    const int lane = threadIdx.x & (kWave - 1);
    const GraphArgs G = graphs[it.graph];
    const int W = G.W;
    const int32_t slot = it.slot0 + lane / W;
    const int64_t rel = static_cast<int64_t>(batch) * G.T + slot;
    const bool active = slot < G.T && rel < l;
    uint64_t steps = 0, h = 0;
    uint32_t err = 0;
    grow_team<kRing>(G, active ? slot : 0, static_cast<uint64_t>(sample_begin + rel), active, seed,
                     lds_path, lds_rec, tree_hash != nullptr, steps, h, err);
    for (int off = W / 2; off > 0; off >>= 1) {
        steps += __shfl_xor(steps, off, kWave);
        h += __shfl_xor(h, off, kWave);
    }
    const bool leader = (lane & (W - 1)) == 0;
    if (active && leader && tree_hash) tree_hash[static_cast<int64_t>(it.graph) * l + rel] = h;
    if (err) atomicOr(status, err);
    const uint64_t wsteps = wave_sum(leader ? steps : 0ull);
    if (lane == 0 && total_steps && wsteps)
        atomicAdd(reinterpret_cast<unsigned long long*>(&total_steps[it.graph]),
                  static_cast<unsigned long long>(wsteps));
}

// One wave per work item: 64 / W trees of one graph, W walkers each (W from the graph).
template <bool kRing>
__global__ void __launch_bounds__(kWave) wilson_team(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                                     int32_t nitems, uint32_t* queue, int32_t batch,
                                                     int64_t sample_begin, int64_t l, uint64_t seed,
                                                     uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    __shared__ uint2 lds_path[kRing ? kPathBuf : 1][kWave];
    __shared__ uint4 lds_rec[4][kWave];
    if (queue == nullptr) {
        if (static_cast<int32_t>(blockIdx.x) < nitems)
            run_team_item<kRing>(graphs, items[blockIdx.x], batch, sample_begin, l, seed, lds_path,
                                 lds_rec, tree_hash, total_steps, status);
        return;
    }
    while (true) {
        uint32_t idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(queue, 1u);
        idx = __shfl(idx, 0, kWave);
        if (idx >= static_cast<uint32_t>(nitems)) break;
        run_team_item<kRing>(graphs, items[idx], batch, sample_begin, l, seed, lds_path, lds_rec,
                             tree_hash, total_steps, status);
    }
}

}  // namespace

int team_resident_waves(bool ring) {
    int per_cu = 0;
    const hipError_t e = ring ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wilson_team<true>, kWave, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wilson_team<false>, kWave, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
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

// Sets every slot of every graph to the fresh state (root in the tree, all else zero).
__global__ void init_state(const GraphArgs* __restrict__ graphs, const int64_t* __restrict__ node_off, int32_t G,
                           int64_t total_nodes) {
    for (int64_t gx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; gx < total_nodes;
         gx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t g = graph_of(node_off, G, gx);
        const GraphArgs A = graphs[g];
        const int64_t x = gx - node_off[g];
        const uint64_t v = (x == A.root) ? kInTree : 0ull;
        for (int32_t t = 0; t < A.T; ++t) A.state[static_cast<int64_t>(t) * A.stride + x] = v;
    }
}

__global__ void zero_outputs(uint64_t* counts, uint64_t* counts_sq, int64_t total_nodes, uint64_t* total_steps,
                             int32_t G, uint32_t* status, uint32_t* queue) {
    const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = tid; i < total_nodes; i += stride) {
        if (counts) counts[i] = 0;
        if (counts_sq) counts_sq[i] = 0;
    }
    for (int64_t i = tid; i < G; i += stride)
        if (total_steps) total_steps[i] = 0;
    if (tid == 0) {
        *status = 0;
        *queue = 0;
    }
}

__global__ void reset_queue(uint32_t* queue) { *queue = 0; }

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
        const bool is_root = (x == A.root);
        for (int d = 0; d < dumps.count; ++d) {
            const uint64_t w = A.state[static_cast<int64_t>(dumps.slot[d]) * A.stride + x];
            parents[static_cast<int64_t>(dumps.out[d]) * A.n + x] = is_root ? -1 : static_cast<int32_t>(st_next(w));
        }
        const uint64_t fresh = is_root ? kInTree : 0ull;
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
        if (counts) counts[gx] += c1;
        if (counts_sq) counts_sq[gx] += c2;
    }
}

// ---------------------------------------------------------------------- planning ------
struct Plan {
    std::vector<int32_t> W, T, S;     // per graph: walkers per tree, tree slots, trees per wave
    std::vector<int64_t> stride;      // per graph: words per slot
    std::vector<int64_t> node_off;
    int64_t total_nodes = 0;
    int32_t batches = 1;
    bool team = false;                // some graph uses more than one walker per tree
};

// Bytes of tree state the automatic plan may use: half of the device's memory (144 GB of the
// 288 GB of an MI355X), so that every tree of BA(10^6) x 10^4 (80 GB) or of R-MAT scale 23 x
// 5000 (133 GB) is in flight at once.  Total, not free, memory keeps the plan identical between
// the workspace query and the call that uses the workspace.
int64_t default_state_budget() {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) {
        (void)hipGetLastError();
        return 96ll << 30;
    }
    return static_cast<int64_t>(total_b / 2);
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
    for (int32_t g = 0; g < G; ++g) {
        if (graphs[g].n < 2 || !graphs[g].row_ptr || !graphs[g].col || !graphs[g].rec || !graphs[g].bfs_order)
            return fail(RWC_ERR_INVALID_ARG, "graph %d is not a built CSR", g);
        plan->node_off[g + 1] = plan->node_off[g] + graphs[g].n;
    }
    plan->total_nodes = plan->node_off[G];
    const int64_t l = p->num_samples;
    int64_t state_words = 0;
    for (int32_t g = 0; g < G; ++g) {
        const int64_t n = graphs[g].n;
        const int W = (p->walkers_per_tree > 0) ? p->walkers_per_tree : auto_walkers(n);
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
        state_words += T * plan->stride[g];
    }
    const int64_t budget = (p->trees_in_flight <= 0) ? default_state_budget() : 0;
    if (p->trees_in_flight <= 0 && state_words * 8 > budget) {
        // shrink every graph's slots by the same factor to fit the automatic budget
        const double f = static_cast<double>(budget) / (8.0 * static_cast<double>(state_words));
        for (int32_t g = 0; g < G; ++g) {
            int64_t T = static_cast<int64_t>(plan->T[g] * f) / plan->S[g] * plan->S[g];
            plan->T[g] = static_cast<int32_t>(T < plan->S[g] ? plan->S[g] : T);
        }
    }
    int32_t batches = 1;
    for (int32_t g = 0; g < G; ++g) {
        const int64_t b = (l + plan->T[g] - 1) / plan->T[g];
        batches = b > batches ? static_cast<int32_t>(b) : batches;
    }
    plan->batches = batches;
    return RWC_OK;
}

struct SampleLayout {
    std::vector<uint64_t*> state;
    GraphArgs* graphs;
    int64_t* node_off;
    Item* items;
    uint32_t* queue;
    uint32_t* status;
    size_t total;
};

int64_t max_items(int32_t G, const Plan& plan) {
    int64_t k = 0;
    for (int32_t g = 0; g < G; ++g) k += (plan.T[g] + plan.S[g] - 1) / plan.S[g];
    return k;
}

SampleLayout carve_sample(void* ws, int32_t G, const Plan& plan) {
    Carver c(ws);
    SampleLayout L{};
    L.state.resize(G);
    for (int32_t g = 0; g < G; ++g) L.state[g] = c.take<uint64_t>(static_cast<size_t>(plan.T[g]) * plan.stride[g]);
    L.graphs = c.take<GraphArgs>(G);
    L.node_off = c.take<int64_t>(G + 1);
    L.items = c.take<Item>(max_items(G, plan));
    L.queue = c.take<uint32_t>(1);
    L.status = c.take<uint32_t>(1);
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

// Private stream for hipGraph capture: begin() orders it after the caller's stream;
// end_and_launch() ends the capture, instantiates and launches the graph, and orders the
// caller's stream after it.
struct CaptureStream {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;

    int begin(hipStream_t caller) {
        RWC_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        RWC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        RWC_HIP(hipEventRecord(ev, caller));
        RWC_HIP(hipStreamWaitEvent(stream, ev, 0));
        RWC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        capturing = true;
        return RWC_OK;
    }
    int end_and_launch(hipStream_t caller, int launch_rc) {
        capturing = false;
        const hipError_t e = hipStreamEndCapture(stream, &graph);
        if (launch_rc != RWC_OK) return launch_rc;
        if (e != hipSuccess) return fail(RWC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        RWC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        RWC_HIP(hipGraphLaunch(exec, stream));
        RWC_HIP(hipEventRecord(ev, stream));
        RWC_HIP(hipStreamWaitEvent(caller, ev, 0));
        return RWC_OK;
    }
    ~CaptureStream() {   // teardown: failures here have nobody to report to
        if (capturing) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev) (void)hipEventDestroy(ev);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

int validate(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p) {
    if (!graphs || !p || G < 1) return fail(RWC_ERR_INVALID_ARG, "graphs/params missing or num_graphs < 1");
    if (p->num_samples < 1) return fail(RWC_ERR_INVALID_ARG, "num_samples must be positive");
    if (p->sample_begin < 0 || p->num_samples > (1ll << 32) || p->sample_begin > (1ll << 32) - p->num_samples)
        return fail(RWC_ERR_INVALID_ARG, "sample indices must lie in [0, 2^32)");
    if (p->root >= 0 && G != 1) return fail(RWC_ERR_INVALID_ARG, "an explicit root needs a single graph");
    if (p->root >= graphs[0].n) return fail(RWC_ERR_INVALID_ARG, "root out of range");
    const int W = p->walkers_per_tree;
    if (W < 0 || W > kWave || (W & (W - 1)) != 0)
        return fail(RWC_ERR_INVALID_ARG, "walkers_per_tree must be 0 (automatic) or a power of two up to 64");
    if ((p->flags & RWC_SAMPLE_SPREAD_STARTS) && (p->flags & RWC_SAMPLE_SHARED_STARTS))
        return fail(RWC_ERR_INVALID_ARG, "spread and shared starts are exclusive");
    if ((p->flags & RWC_SAMPLE_PATH_RING) && (p->flags & RWC_SAMPLE_NO_PATH_RING))
        return fail(RWC_ERR_INVALID_ARG, "path ring and no path ring are exclusive");
    if ((p->flags & RWC_SAMPLE_BFS_STARTS) && (p->flags & RWC_SAMPLE_ID_STARTS))
        return fail(RWC_ERR_INVALID_ARG, "breadth-first and ascending starts are exclusive");
    return RWC_OK;
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
    *bytes = carve_sample(nullptr, num_graphs, plan).total;
    return RWC_OK;
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
    if (capture && out->timing_ms)
        return fail(RWC_ERR_INVALID_ARG, "timing_ms is not available with RWC_SAMPLE_GRAPH_CAPTURE");
    Plan plan;
    RWC_CHECK(make_plan(graphs, G, p, &plan));
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_sample(nullptr, G, plan).total));
    SampleLayout L = carve_sample(ws, G, plan);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t l = p->num_samples;

    std::vector<GraphArgs> hg(G);
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
        hg[g].state = L.state[g];
        hg[g].stride = plan.stride[g];
        hg[g].guard = steps;
        hg[g].n = graphs[g].n;
        hg[g].root = (p->root >= 0) ? p->root : graphs[g].pivot;
        hg[g].graph_word = p->graph_index_base + static_cast<uint32_t>(g);
        hg[g].T = plan.T[g];
        hg[g].W = plan.W[g];
        hg[g].spread = spread_starts(graphs[g], p->flags) ? 1 : 0;
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
    const bool fills = plan.team && 3 * max_items(G, plan) >= 2 * resident;
    // Start order, measured: breadth-first starts make batches of many meshes (spread starts)
    // a third faster (256 mixed graphs: 4.5 -> 3.0 s, their 128 grids alone 4.0 -> 3.1 s) but
    // every single graph slower, meshes included (a 25 k-node grid with 50 000 trees: 10 %, a
    // 97 k-node grid with 2000-20 000 trees: 5-15 %), and small-world graphs (shared starts)
    // by much more.  So they are taken for the meshes of calls with several graphs and a queue
    // of at least twice the resident waves.
    const bool queued = plan.team && G > 1 && max_items(G, plan) >= 2 * resident;
    for (int32_t g = 0; g < G; ++g) {
        const bool bfs = (p->flags & RWC_SAMPLE_BFS_STARTS) ||
                         (!(p->flags & RWC_SAMPLE_ID_STARTS) && queued && plan.W[g] > 1 && hg[g].spread);
        hg[g].order = bfs ? graphs[g].bfs_order : nullptr;
    }
    const bool ring = (p->flags & RWC_SAMPLE_PATH_RING) ? true
                      : (p->flags & RWC_SAMPLE_NO_PATH_RING) ? false
                                                              : (any_spread || !any_dense_weighted || !fills);
    // Work items with the longest trees first: a tree's time grows with n / W.
    std::vector<int32_t> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return static_cast<int64_t>(graphs[a].n) * plan.W[b] > static_cast<int64_t>(graphs[b].n) * plan.W[a];
    });
    std::vector<Item> items;
    items.reserve(max_items(G, plan));
    for (int32_t g : order)
        for (int32_t s0 = 0; s0 < plan.T[g]; s0 += plan.S[g]) items.push_back(Item{g, s0});
    RWC_HIP(hipMemcpyAsync(L.graphs, hg.data(), sizeof(GraphArgs) * G, hipMemcpyHostToDevice, s));
    RWC_HIP(hipMemcpyAsync(L.node_off, plan.node_off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    RWC_HIP(hipMemcpyAsync(L.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice, s));

    const bool persistent = (p->flags & RWC_SAMPLE_PERSISTENT) != 0;
    const WalkKernel walk = !plan.team ? static_cast<WalkKernel>(wilson_walk)
                            : ring     ? static_cast<WalkKernel>(wilson_team<true>)
                                       : static_cast<WalkKernel>(wilson_team<false>);
    int grid_persistent = 0;
    if (persistent) {
        int per_cu = 0;
        RWC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, walk, kWave, 0));
        if (per_cu < 1) per_cu = 1;
        grid_persistent = per_cu * device_cu_count();
    }
    Timer timer;
    if (out->timing_ms) RWC_CHECK(timer.init());
    // A capture runs on a private stream (the caller's may be the legacy default stream,
    // which cannot be captured), ordered after and before the caller's stream by events.
    CaptureStream cap;
    if (capture) RWC_CHECK(cap.begin(s));
    const hipStream_t ls = capture ? cap.stream : s;
    const int32_t nit = static_cast<int32_t>(items.size());

    auto launches = [&]() -> int {
        const unsigned node_blocks = blocks_for(plan.total_nodes, 256) < 8192 ? blocks_for(plan.total_nodes, 256) : 8192;
        const bool accumulate = (p->flags & RWC_SAMPLE_ACCUMULATE) != 0;
        hipLaunchKernelGGL(zero_outputs, dim3(node_blocks), dim3(256), 0, ls, accumulate ? nullptr : out->counts,
                           accumulate ? nullptr : out->counts_sq, plan.total_nodes,
                           accumulate ? nullptr : out->total_steps, G, L.status, L.queue);
        hipLaunchKernelGGL(init_state, dim3(node_blocks), dim3(256), 0, ls, L.graphs, L.node_off, G, plan.total_nodes);
        for (int32_t b = 0; b < plan.batches; ++b) {
            // every graph runs its samples [b*T_g, (b+1)*T_g); graphs with fewer batches idle
            if (out->timing_ms) RWC_HIP(hipEventRecord(timer.ev[0], ls));
            if (persistent) {
                hipLaunchKernelGGL(reset_queue, dim3(1), dim3(1), 0, ls, L.queue);
                const int grid = grid_persistent < nit ? grid_persistent : nit;
                hipLaunchKernelGGL(walk, dim3(grid), dim3(kWave), 0, ls, L.graphs, L.items, nit, L.queue, b,
                                   p->sample_begin, l, p->seed, out->tree_hash, out->total_steps, L.status);
            } else {
                hipLaunchKernelGGL(walk, dim3(nit), dim3(kWave), 0, ls, L.graphs, L.items, nit, nullptr, b,
                                   p->sample_begin, l, p->seed, out->tree_hash, out->total_steps, L.status);
            }
            DumpArgs dumps{};
            for (int d = 0; d < out->ndump; ++d) {
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

    int rc = launches();
    if (capture) {
        const int rc2 = cap.end_and_launch(s, rc);
        RWC_CHECK(rc);
        RWC_CHECK(rc2);
    }
    RWC_CHECK(rc);
    uint32_t status = 0;
    RWC_HIP(hipMemcpyAsync(&status, L.status, sizeof(status), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    if (out->timing_ms) {
        out->timing_ms[0] = timer.walk_ms;
        out->timing_ms[1] = timer.reduce_ms;
    }
    if (out->plan) {
        // graph 0's plan (every graph's plan is the same unless chosen automatically)
        out->plan[0] = plan.W[0];
        out->plan[1] = plan.T[0];
        out->plan[2] = plan.batches;
        out->plan[3] = !plan.team ? 0 : (ring ? 2 : 1);
        out->plan[4] = hg[0].spread;
        out->plan[5] = hg[0].order != nullptr ? 1 : 0;
    }
    return device_error_to_status(status);
}
