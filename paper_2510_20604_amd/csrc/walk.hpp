// The walk kernels of rwc_sample_forests: Wilson's algorithm (Section 5, Algorithm 3), one
// lane per tree (wilson_walk) or a team of lanes per tree (wilson_team), with the argument
// tables they read.  Included by sampler.hip, which plans and launches them.
//
// RandomNeighbor(u) at the k-th departure from u in sample i of graph word g is
// Philox4x32-10((k, u, i, g), seed), optionally placed in its stratum (stratified_word), with
// u the node's input id (record word kRecId); the kernels address memory by internal index.  A
// node's successive choices are therefore fixed in advance, which makes the tree and every
// count independent of the order in which walks are run (cycle popping), so results match the
// serial order of Algorithm 3 exactly.
#pragma once

#include "common.hpp"
#include "device.hpp"
#include "select.hpp"

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
    const int32_t* node_id;     // input id of each internal index (keys, checksums, outputs)
    const int32_t* node_index;  // internal index of each input id
    const uint32_t* rootmask;   // bitmap of the root set (n bits, internal indices), or null:
                                // the root is `root` (an internal index)
    int32_t n;
    int32_t root;
    uint32_t graph_word;
    int32_t T;              // tree slots (trees in flight) of this graph
    int32_t W;              // walkers per tree
    int32_t spread;         // each walker of a team takes starts from its own range
    Strata strata;          // stack entries stratified over the call's samples (count >= 2)
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

// Grows the tree of slot `slot` for absolute sample `sample` (one lane).  kStrat: stack
// entries stratified over the call's samples (stratified_word).
template <bool kStrat>
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
            const uint32_t xid = rec_word(ra, rb, rc, rd, kRecId);
            uint64_t r = philox_x64(k, xid, sw, gw, k0, k1);
            if constexpr (kStrat) r = stratified_word(r, k, xid, sw, gw, k0, k1, G.strata);
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
                if (want_hash) h += splitmix64((static_cast<uint64_t>(G.node_id[x]) << 32) | G.node_id[p]);
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
template <bool kStrat>
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
    if (active)
        grow_tree<kStrat>(G, slot, static_cast<uint64_t>(sample_begin + rel), seed, tree_hash != nullptr, steps, h,
                          err);
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
template <bool kStrat>
__device__ __forceinline__ void walk_items(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                           int32_t nitems, uint32_t* queue, int32_t batch, int64_t sample_begin,
                                           int64_t l, uint64_t seed, uint64_t* tree_hash, uint64_t* total_steps,
                                           uint32_t* status) {
    if (queue == nullptr) {
        if (static_cast<int32_t>(blockIdx.x) < nitems)
            run_item<kStrat>(graphs, items[blockIdx.x], batch, sample_begin, l, seed, tree_hash, total_steps, status);
        return;
    }
    while (true) {
        uint32_t idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(queue, 1u);
        idx = __shfl(idx, 0, kWave);
        if (idx >= static_cast<uint32_t>(nitems)) break;
        run_item<kStrat>(graphs, items[idx], batch, sample_begin, l, seed, tree_hash, total_steps, status);
    }
}

__global__ void __launch_bounds__(kWave) wilson_walk(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                                     int32_t nitems, uint32_t* queue, int32_t batch,
                                                     int64_t sample_begin, int64_t l, uint64_t seed,
                                                     uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    walk_items<false>(graphs, items, nitems, queue, batch, sample_begin, l, seed, tree_hash, total_steps, status);
}

// The same with stratified stack entries (a kernel of its own, so that the plain walk keeps
// its register budget).
__global__ void __launch_bounds__(kWave)
    wilson_walk_strata(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items, int32_t nitems,
                       uint32_t* queue, int32_t batch, int64_t sample_begin, int64_t l, uint64_t seed,
                       uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    walk_items<true>(graphs, items, nitems, queue, batch, sample_begin, l, seed, tree_hash, total_steps, status);
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

// The same accesses on tree state held in LDS (small graphs: all n words of a tree fit in the
// work-group's LDS), where they are ds_read / ds_write / ds_cmpst instructions.
__device__ __forceinline__ uint64_t st_load(const RWC_LDS uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_store(RWC_LDS uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool st_cas(RWC_LDS uint64_t* p, uint64_t expected, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
}

// st: the tree's state words, in HBM (RWC_GLOBAL uint64_t*) or in LDS (RWC_LDS uint64_t*).
template <bool kRing, bool kStrat, class StatePtr>
__device__ void grow_team(const GraphArgs& G, StatePtr st, uint64_t sample, bool active, uint64_t seed,
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
            const uint32_t hid = rec_at(kRecId);   // the head's input id keys its stack
            uint64_t r = philox_x64(k, hid, sw, gw, k0, k1);
            if constexpr (kStrat) r = stratified_word(r, k, hid, sw, gw, k0, k1, G.strata);
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
                if (want_hash)
                    hsum += splitmix64((static_cast<uint64_t>(G.node_id[c]) << 32) | G.node_id[st_next(w)]);
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
                        hsum += splitmix64((static_cast<uint64_t>(G.node_id[buf(d)]) << 32) |
                                           G.node_id[d == 0 ? act_v : buf(d - 1)]);
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

template <bool kRing, bool kStrat>
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
    grow_team<kRing, kStrat>(G, global_ptr(G.state + static_cast<int64_t>(active ? slot : 0) * G.stride),
                     static_cast<uint64_t>(sample_begin + rel), active, seed, lds_path, lds_rec, tree_hash != nullptr,
                     steps, h, err);
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
template <bool kRing, bool kStrat>
__device__ __forceinline__ void team_items(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                           int32_t nitems, uint32_t* queue, int32_t batch, int64_t sample_begin,
                                           int64_t l, uint64_t seed, uint2 (*lds_path)[kWave],
                                           uint4 (*lds_rec)[kWave], uint64_t* tree_hash, uint64_t* total_steps,
                                           uint32_t* status) {
    if (queue == nullptr) {
        if (static_cast<int32_t>(blockIdx.x) < nitems)
            run_team_item<kRing, kStrat>(graphs, items[blockIdx.x], batch, sample_begin, l, seed, lds_path,
                                         lds_rec, tree_hash, total_steps, status);
        return;
    }
    while (true) {
        uint32_t idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(queue, 1u);
        idx = __shfl(idx, 0, kWave);
        if (idx >= static_cast<uint32_t>(nitems)) break;
        run_team_item<kRing, kStrat>(graphs, items[idx], batch, sample_begin, l, seed, lds_path, lds_rec,
                                     tree_hash, total_steps, status);
    }
}

template <bool kRing>
__global__ void __launch_bounds__(kWave) wilson_team(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                                     int32_t nitems, uint32_t* queue, int32_t batch,
                                                     int64_t sample_begin, int64_t l, uint64_t seed,
                                                     uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    __shared__ uint2 lds_path[kRing ? kPathBuf : 1][kWave];
    __shared__ uint4 lds_rec[4][kWave];
    team_items<kRing, false>(graphs, items, nitems, queue, batch, sample_begin, l, seed, lds_path, lds_rec,
                             tree_hash, total_steps, status);
}

template <bool kRing>
__global__ void __launch_bounds__(kWave)
    wilson_team_strata(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items, int32_t nitems,
                       uint32_t* queue, int32_t batch, int64_t sample_begin, int64_t l, uint64_t seed,
                       uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    __shared__ uint2 lds_path[kRing ? kPathBuf : 1][kWave];
    __shared__ uint4 lds_rec[4][kWave];
    team_items<kRing, true>(graphs, items, nitems, queue, batch, sample_begin, l, seed, lds_path, lds_rec,
                            tree_hash, total_steps, status);
}

// ---------------------------------------------------------------------------------------
// LDS-resident trees.  For a graph whose state words fit in the work-group's LDS (64 / W trees
// of n words each), a wave grows its trees entirely in LDS: the team protocol above is the
// same, but every state access is an LDS operation instead of a random HBM line, and the trees
// need no slots in HBM.  Each work item is a block of 64 / W consecutive samples; the wave
// clears its LDS trees, grows them, then adds every node's departure count (and its square)
// into the call's totals with one atomic per node and writes any requested parent dump.
// ---------------------------------------------------------------------------------------
template <bool kRing, bool kStrat>
__device__ __forceinline__ void run_team_item_lds(const GraphArgs* __restrict__ graphs, const Item it,
                                                  int64_t sample_begin, int64_t l, uint64_t seed,
                                                  uint2 (*lds_path)[kWave], uint4 (*lds_rec)[kWave],
                                                  RWC_LDS uint64_t* lds_state, const int64_t* __restrict__ node_off,
                                                  uint64_t* __restrict__ counts, uint64_t* __restrict__ counts_sq,
                                                  int32_t* __restrict__ parents, const DumpArgs& dumps,
                                                  uint64_t* __restrict__ tree_hash,
                                                  uint64_t* __restrict__ total_steps, uint32_t* __restrict__ status) {
    const int lane = threadIdx.x & (kWave - 1);
    const GraphArgs G = graphs[it.graph];
    const int W = G.W;
    const int team = lane / W;
    const uint32_t tl = static_cast<uint32_t>(lane & (W - 1));
    const int64_t rel = static_cast<int64_t>(it.slot0) + team;   // sample index within the call
    const bool active = rel < l;
    const int32_t n = G.n;
    RWC_LDS uint64_t* st = lds_state + static_cast<int64_t>(team) * G.stride;
    auto is_root = [&](int32_t x) {
        return G.rootmask ? ((G.rootmask[x >> 5] >> (x & 31)) & 1u) != 0 : x == G.root;
    };
    for (int32_t x = static_cast<int32_t>(tl); x < n; x += W) st[x] = is_root(x) ? kInTree : 0ull;
    __syncthreads();
    uint64_t steps = 0, h = 0;
    uint32_t err = 0;
    grow_team<kRing, kStrat>(G, st, static_cast<uint64_t>(sample_begin + rel), active, seed, lds_path, lds_rec,
                             tree_hash != nullptr, steps, h, err);
    __syncthreads();
    if (active) {
        const int64_t off = node_off[it.graph];
        int32_t dump_out = -1;
        for (int d = 0; d < dumps.count; ++d)
            if (dumps.slot[d] == rel) dump_out = dumps.out[d];
        for (int32_t x = static_cast<int32_t>(tl); x < n; x += W) {
            const uint64_t w = st[x];
            const uint32_t c = st_cnt(w);
            const int64_t id = G.node_id[x];   // outputs are indexed by input id
            if (c) {
                atomicAdd(reinterpret_cast<unsigned long long*>(&counts[off + id]), static_cast<unsigned long long>(c));
                if (counts_sq)
                    atomicAdd(reinterpret_cast<unsigned long long*>(&counts_sq[off + id]),
                              static_cast<unsigned long long>(square_count(c)));
            }
            if (dump_out >= 0)
                parents[static_cast<int64_t>(dump_out) * n + id] = is_root(x) ? -1 : G.node_id[st_next(w)];
        }
    }
    for (int off = W / 2; off > 0; off >>= 1) {
        steps += __shfl_xor(steps, off, kWave);
        h += __shfl_xor(h, off, kWave);
    }
    const bool leader = tl == 0;
    if (active && leader && tree_hash) tree_hash[static_cast<int64_t>(it.graph) * l + rel] = h;
    if (err) atomicOr(status, err);
    const uint64_t wsteps = wave_sum(leader ? steps : 0ull);
    if (lane == 0 && total_steps && wsteps)
        atomicAdd(reinterpret_cast<unsigned long long*>(&total_steps[it.graph]),
                  static_cast<unsigned long long>(wsteps));
    __syncthreads();   // the next item's clearing must not overtake this item's reads
}

// Persistent: a grid of resident waves pops items (graph, first sample) from `queue`.  The
// dynamic LDS holds the state words of 64 / W trees of the largest graph of the call.
template <bool kRing, bool kStrat>
__device__ __forceinline__ void team_items_lds(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items,
                                               int32_t nitems, uint32_t* queue, int64_t sample_begin, int64_t l,
                                               uint64_t seed, const int64_t* __restrict__ node_off, uint64_t* counts,
                                               uint64_t* counts_sq, int32_t* parents, const DumpArgs& dumps,
                                               uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status,
                                               uint2 (*lds_path)[kWave], uint4 (*lds_rec)[kWave],
                                               RWC_LDS uint64_t* lds_state) {
    while (true) {
        uint32_t idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(queue, 1u);
        idx = __shfl(idx, 0, kWave);
        if (idx >= static_cast<uint32_t>(nitems)) break;
        run_team_item_lds<kRing, kStrat>(graphs, items[idx], sample_begin, l, seed, lds_path, lds_rec, lds_state,
                                         node_off, counts, counts_sq, parents, dumps, tree_hash, total_steps, status);
    }
}

template <bool kRing>
__global__ void __launch_bounds__(kWave) wilson_team_lds(const GraphArgs* __restrict__ graphs,
                                                         const Item* __restrict__ items, int32_t nitems, uint32_t* queue,
                                                         int64_t sample_begin, int64_t l, uint64_t seed,
                                                         const int64_t* __restrict__ node_off, uint64_t* counts,
                                                         uint64_t* counts_sq, int32_t* parents, DumpArgs dumps,
                                                         uint64_t* tree_hash, uint64_t* total_steps, uint32_t* status) {
    __shared__ uint2 lds_path[kRing ? kPathBuf : 1][kWave];
    __shared__ uint4 lds_rec[4][kWave];
    extern __shared__ uint64_t lds_state_raw[];
    team_items_lds<kRing, false>(graphs, items, nitems, queue, sample_begin, l, seed, node_off, counts, counts_sq,
                                 parents, dumps, tree_hash, total_steps, status, lds_path, lds_rec,
                                 (RWC_LDS uint64_t*)lds_state_raw);
}

template <bool kRing>
__global__ void __launch_bounds__(kWave)
    wilson_team_lds_strata(const GraphArgs* __restrict__ graphs, const Item* __restrict__ items, int32_t nitems,
                           uint32_t* queue, int64_t sample_begin, int64_t l, uint64_t seed,
                           const int64_t* __restrict__ node_off, uint64_t* counts, uint64_t* counts_sq,
                           int32_t* parents, DumpArgs dumps, uint64_t* tree_hash, uint64_t* total_steps,
                           uint32_t* status) {
    __shared__ uint2 lds_path[kRing ? kPathBuf : 1][kWave];
    __shared__ uint4 lds_rec[4][kWave];
    extern __shared__ uint64_t lds_state_raw[];
    team_items_lds<kRing, true>(graphs, items, nitems, queue, sample_begin, l, seed, node_off, counts, counts_sq,
                                parents, dumps, tree_hash, total_steps, status, lds_path, lds_rec,
                                (RWC_LDS uint64_t*)lds_state_raw);
}

}  // namespace
}  // namespace rwc
