// rwc_build_csr: edge list -> symmetric CSR with sorted rows, integer CDF rows, weighted
// degrees, vol, pivot and a connectivity check, all on the GPU.
//
// Internal order.  On a graph with a heavy degree tail (largest degree above four times the
// mean) nodes are stored by descending weighted degree, ties by ascending input id, so the
// pivot is internal index 0 and the nodes a random walk visits most share cache lines: their
// per-tree state words, records and rows (R-MAT scale 23: the walk 20 % faster).  Otherwise
// the internal order is the input order.  Only memory placement changes: the records carry
// each node's input id, rows list neighbours by ascending input id, and everything the caller
// sees is indexed by input id, so every result is the same in either order.
//
// Rows are produced by an LSD radix sort of the 2m directed entries keyed (internal row << 32 |
// input id of the neighbour), which makes the CSR a deterministic function of the edge set
// (independent of atomics order).  Connectivity uses a lock-free union-find over the input edges: roots are always
// hooked from the larger id to the smaller one with a compare-and-swap, so every parent
// pointer decreases and every find terminates.
#include <utility>

#include "common.hpp"
#include "device.hpp"

namespace rwc {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

struct BuildScalars {
    uint32_t status;
    int32_t max_deg;
    int32_t pivot;        // internal index
    int32_t nroots;
    uint64_t max_s;
    uint64_t vol_fixed;
    uint64_t max_s_in;    // largest weighted degree (fixed point) before the CSR exists
    int32_t max_deg_in;   // largest degree counted from the edge list
    int32_t pivot_id;     // input id of the pivot
};

// ------------------------------------------------------------------ exclusive scan -----
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* total) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wave_tot[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const uint32_t s = wave_tot[w];
        if (w < wid) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Blocked arrangement: thread t owns elements [t*kItems, (t+1)*kItems) of its tile.
__global__ void scan_tile_sums(const uint32_t* __restrict__ in, int64_t len, uint32_t* __restrict__ sums) {
    __shared__ uint32_t wave_tot[kBlock / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile + threadIdx.x * kItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < len) s += in[base + i];
    uint32_t tot;
    block_exclusive_scan(s, wave_tot, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of `count` tile sums in place by one block, chunk by chunk with a carry.
__global__ void scan_sums_single(uint32_t* __restrict__ sums, int64_t count) {
    __shared__ uint32_t wave_tot[kBlock / kWave];
    uint32_t carry = 0;
    for (int64_t c = 0; c < count; c += kTile) {
        const int64_t base = c + threadIdx.x * kItems;
        uint32_t v[kItems];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            v[i] = (base + i < count) ? sums[base + i] : 0u;
            s += v[i];
        }
        uint32_t tot;
        uint32_t pre = block_exclusive_scan(s, wave_tot, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            if (base + i < count) sums[base + i] = pre;
            pre += v[i];
        }
        carry += tot;
    }
}

__global__ void scan_tile_apply(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t len,
                                const uint32_t* __restrict__ sums) {
    __shared__ uint32_t wave_tot[kBlock / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile + threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < len) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, wave_tot, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (base + i < len) out[base + i] = pre;
        pre += v[i];
    }
}

// Exclusive scan of len uint32 values (in may equal out).  `sums` needs
// ceil(len / kTile) entries.
int exclusive_scan(const uint32_t* in, uint32_t* out, int64_t len, uint32_t* sums, hipStream_t s) {
    if (len <= 0) return RWC_OK;
    const unsigned nb = blocks_for(len, kTile);
    hipLaunchKernelGGL(scan_tile_sums, dim3(nb), dim3(kBlock), 0, s, in, len, sums);
    hipLaunchKernelGGL(scan_sums_single, dim3(1), dim3(kBlock), 0, s, sums, static_cast<int64_t>(nb));
    hipLaunchKernelGGL(scan_tile_apply, dim3(nb), dim3(kBlock), 0, s, in, out, len, sums);
    RWC_HIP(hipGetLastError());
    return RWC_OK;
}

// --------------------------------------------------------------- LSD radix sort -------
// Striped arrangement: in round r thread t handles element r*kBlock + t of its tile, so the
// element order within a tile is (round, thread) and ranks computed in that order are
// stable.
__global__ void radix_hist(const uint64_t* __restrict__ keys, int64_t len, int shift,
                           uint32_t* __restrict__ ghist, int nb) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kTile;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = tile0 + r * kBlock + threadIdx.x;
        if (i < len) atomicAdd(&hist[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    ghist[static_cast<int64_t>(threadIdx.x) * nb + blockIdx.x] = hist[threadIdx.x];
}

__global__ void radix_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                              uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t len,
                              int shift, const uint32_t* __restrict__ goff, int nb) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kBlock / kWave][256];
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    base[t] = goff[static_cast<int64_t>(t) * nb + blockIdx.x];
    run[t] = 0;
    const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int r = 0; r < kItems; ++r) {
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) wcnt[w][t] = 0;
        __syncthreads();
        const int64_t i = tile0 + r * kBlock + t;
        const bool valid = i < len;
        const uint64_t k = valid ? kin[i] : 0ull;
        const int32_t v = valid ? vin[i] : 0;
        const uint32_t d = static_cast<uint32_t>(k >> shift) & 0xFFu;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const uint32_t rank = __popcll(same & lt_mask);
        if (valid && rank == 0) wcnt[wid][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d];
            for (int w = 0; w < wid; ++w) off += wcnt[w][d];
            const int64_t pos = static_cast<int64_t>(base[d]) + off + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) add += wcnt[w][t];
        run[t] += add;
    }
}

// ----------------------------------------------------------------- build kernels ------
__global__ void init_scalars(BuildScalars* sc) {
    sc->status = 0;
    sc->max_deg = 0;
    sc->pivot = 0x7FFFFFFF;
    sc->nroots = 0;
    sc->max_s = 0;
    sc->vol_fixed = 0;
    sc->max_s_in = 0;
    sc->max_deg_in = 0;
    sc->pivot_id = -1;
}

__global__ void fill_u32(uint32_t* p, int64_t len, uint32_t v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void validate_edges(int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                               const float* __restrict__ w, int32_t n, BuildScalars* sc) {
    uint32_t bits = 0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        if (a < 0 || a >= n || b < 0 || b >= n) bits |= kErrNodeRange;
        if (a == b) bits |= kErrSelfLoop;
        if (w) {
            const float x = w[e];
            // NaN fails both comparisons
            if (!(x >= 0.5f && x < 65536.0f)) bits |= kErrWeight;
        }
    }
    if (bits) atomicOr(&sc->status, bits);
}

__global__ void count_degrees(int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                              int32_t n, uint32_t* __restrict__ deg) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        if (a >= 0 && a < n && b >= 0 && b < n) {
            atomicAdd(&deg[a], 1u);
            atomicAdd(&deg[b], 1u);
        }
    }
}

// Weighted degree of every input id, fixed point (w 2^24 is an exact integer; the sums are
// exact and independent of the order of the atomics), with the largest degree and strength.
__global__ void strength_in(int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                            const float* __restrict__ w, uint64_t* __restrict__ sfix) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const unsigned long long W = static_cast<unsigned long long>(static_cast<double>(w[e]) * 16777216.0);
        atomicAdd(reinterpret_cast<unsigned long long*>(&sfix[src[e]]), W);
        atomicAdd(reinterpret_cast<unsigned long long*>(&sfix[dst[e]]), W);
    }
}

__global__ void degree_stats(int32_t n, const uint32_t* __restrict__ deg, uint64_t* __restrict__ sfix, bool weighted,
                             BuildScalars* sc) {
    uint64_t ms = 0;
    int32_t md = 0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (!weighted) sfix[u] = static_cast<uint64_t>(deg[u]) << 24;
        ms = sfix[u] > ms ? sfix[u] : ms;
        md = static_cast<int32_t>(deg[u]) > md ? static_cast<int32_t>(deg[u]) : md;
    }
    if (ms) atomicMax(reinterpret_cast<unsigned long long*>(&sc->max_s_in), static_cast<unsigned long long>(ms));
    if (md) atomicMax(&sc->max_deg_in, md);
}

// Sort keys of the internal order: the strength below the largest (ascending key = descending
// strength), the input id as value; the stable sort keeps ties in ascending id.
__global__ void order_keys(int32_t n, const uint64_t* __restrict__ sfix, const BuildScalars* __restrict__ sc,
                           uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const uint64_t top = sc->max_s_in;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        keys[u] = top - sfix[u];
        vals[u] = static_cast<int32_t>(u);
    }
}

__global__ void identity_order(int32_t n, int32_t* __restrict__ node_id) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        node_id[u] = static_cast<int32_t>(u);
}

// node_index = inverse of node_id; degrees in internal order (the scan input for row_ptr).
__global__ void invert_order(int32_t n, const int32_t* __restrict__ node_id, int32_t* __restrict__ node_index,
                             const uint32_t* __restrict__ deg_in, uint32_t* __restrict__ deg) {
    for (int64_t x = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; x < n;
         x += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t id = node_id[x];
        node_index[id] = static_cast<int32_t>(x);
        deg[x] = deg_in[id];
    }
}

__global__ void make_keys(int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                          const int32_t* __restrict__ node_index, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ vals) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t a = static_cast<uint32_t>(src[e]), b = static_cast<uint32_t>(dst[e]);
        const uint64_t xa = static_cast<uint32_t>(node_index[a]), xb = static_cast<uint32_t>(node_index[b]);
        keys[2 * e] = (xa << 32) | b;
        keys[2 * e + 1] = (xb << 32) | a;
        vals[2 * e] = static_cast<int32_t>(2 * e);
        vals[2 * e + 1] = static_cast<int32_t>(2 * e + 1);
    }
}

__global__ void fill_csr(int64_t nnz, const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                         const float* __restrict__ w, const int32_t* __restrict__ node_index, int32_t* __restrict__ col,
                         int32_t* __restrict__ edge_id, float* __restrict__ weight, BuildScalars* sc) {
    uint32_t bits = 0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nnz;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t k = keys[i];
        col[i] = node_index[static_cast<uint32_t>(k)];
        const int32_t e = vals[i] >> 1;
        edge_id[i] = e;
        weight[i] = w ? w[e] : 1.0f;
        if (i > 0 && keys[i - 1] == k) bits |= kErrDupEdge;
    }
    if (bits) atomicOr(&sc->status, bits);
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x, int lane) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x;
}

// One wave per row (grid-stride over rows): integer CDF, strength, and per-wave partial
// reductions of vol, max degree and max strength.
__global__ void row_pass(int32_t n, const int32_t* __restrict__ row_ptr, const float* __restrict__ weight,
                         uint64_t* __restrict__ cdf, double* __restrict__ strength, uint64_t* __restrict__ sfix,
                         BuildScalars* sc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
    uint64_t vol = 0, maxs = 0;
    int32_t maxdeg = 0;
    uint32_t bits = 0;
    for (int64_t u = wave; u < n; u += nwaves) {
        const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
        uint64_t S;
        if (cdf) {
            uint64_t carry = 0;
            for (int32_t b0 = beg; b0 < end; b0 += kWave) {
                const int32_t i = b0 + lane;
                // weight is a float32 in [0.5, 65536): w * 2^24 is an exact integer below 2^40
                const uint64_t W = (i < end) ? static_cast<uint64_t>(static_cast<double>(weight[i]) * 16777216.0) : 0ull;
                const uint64_t x = wave_incl_scan_u64(W, lane);   // < 64 * 2^40, no wrap
                if (i < end) cdf[i] = carry + x;
                // saturate at 2^63: a row above 2^53 is rejected below, and a long row of
                // large weights must not wrap back under that bound first
                const uint64_t chunk = __shfl(x, kWave - 1, kWave);
                carry = (carry >= (1ull << 63) - chunk) ? (1ull << 63) : carry + chunk;
            }
            S = carry;
        } else {
            S = static_cast<uint64_t>(end - beg) << 24;
        }
        if (lane == 0) {
            if (S >= (1ull << 53)) bits |= kErrStrength;
            strength[u] = static_cast<double>(S) * (1.0 / 16777216.0);
            sfix[u] = S;
            // vol must stay an exact uint64: every row is below 2^63 here, so a wrap of the
            // running sum is seen as a result smaller than the row added
            if (vol + S < vol) bits |= kErrVolume;
            vol += S;
            maxs = S > maxs ? S : maxs;
            maxdeg = (end - beg) > maxdeg ? (end - beg) : maxdeg;
        }
    }
    if (lane == 0) {
        if (vol) {
            const uint64_t before = atomicAdd(reinterpret_cast<unsigned long long*>(&sc->vol_fixed),
                                              static_cast<unsigned long long>(vol));
            if (before + vol < before) bits |= kErrVolume;   // the total wrapped past 2^64
        }
        if (maxs) atomicMax(reinterpret_cast<unsigned long long*>(&sc->max_s), static_cast<unsigned long long>(maxs));
        if (maxdeg) atomicMax(&sc->max_deg, maxdeg);
        if (bits) atomicOr(&sc->status, bits);
    }
}

// 64-byte node records (layout in device.hpp): one aligned load gives a walker the degree, the
// row offset and the row's first neighbours (with their CDF values and the row's total when
// weighted).
__global__ void build_records(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                              const uint64_t* __restrict__ cdf, const int32_t* __restrict__ node_id,
                              uint32_t* __restrict__ rec) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t beg = row_ptr[u], deg = row_ptr[u + 1] - beg;
        uint32_t r[kRecWords];
#pragma unroll
        for (int i = 0; i < kRecWords; ++i) r[i] = 0;
        r[0] = static_cast<uint32_t>(deg);
        r[1] = static_cast<uint32_t>(beg);
        r[kRecId] = static_cast<uint32_t>(node_id[u]);
        if (cdf) {
#pragma unroll
            for (int i = 0; i < kRecInlineWeighted; ++i) {
                if (i < deg) {
                    r[kRecFirst + i] = static_cast<uint32_t>(col[beg + i]);
                    const uint64_t c = cdf[beg + i];
                    r[8 + 2 * i] = static_cast<uint32_t>(c);
                    r[9 + 2 * i] = static_cast<uint32_t>(c >> 32);
                }
            }
            if (deg > 0) {
                const uint64_t total = cdf[beg + deg - 1];
                r[6] = static_cast<uint32_t>(total);
                r[7] = static_cast<uint32_t>(total >> 32);
            }
        } else {
#pragma unroll
            for (int i = 0; i < kRecInline; ++i)
                if (i < deg) r[kRecFirst + i] = static_cast<uint32_t>(col[beg + i]);
        }
        uint4* out = reinterpret_cast<uint4*>(rec + static_cast<int64_t>(kRecWords) * u);
#pragma unroll
        for (int q = 0; q < kRecWords / 4; ++q) out[q] = make_uint4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
    }
}

__global__ void pick_pivot(int32_t n, const uint64_t* __restrict__ sfix, BuildScalars* sc) {
    const uint64_t target = sc->max_s;
    int32_t best = 0x7FFFFFFF;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (sfix[u] == target && u < best) best = static_cast<int32_t>(u);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int32_t o = __shfl_xor(best, off, kWave);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && best != 0x7FFFFFFF) atomicMin(&sc->pivot, best);
}

__global__ void pivot_input_id(const int32_t* __restrict__ node_id, BuildScalars* sc) {
    const int32_t p = sc->pivot;
    if (p != 0x7FFFFFFF) sc->pivot_id = node_id[p];
}

// Breadth-first order from the pivot, built in place: order[0..tail) is the queue; each level
// expands order[lo, hi) and appends newly reached nodes.  The order within a level follows
// the atomics and is not reproducible; nothing that depends on it is observable except speed
// (any start order yields the same forest).

// The frontier bounds live on the device, so that levels can be launched back to back without a
// host round trip each: the current level expands order[lo, hi); bfs_advance then moves to the
// nodes appended meanwhile and stops the search (done) once a level adds nothing.
constexpr int32_t kBfsLongRow = 4096;   // frontier rows longer than this are shared by every wave
constexpr int kBfsLongRows = 256;       // such rows one level defers (any more expand in place)

struct BfsState {
    uint32_t tail;    // nodes in the queue so far
    uint32_t lo, hi;  // the current level's frontier
    int32_t level;    // its distance from the pivot
    int32_t done;     // no frontier left: further launches return at once
    int32_t depth;    // largest distance reached
    uint32_t nlong;   // long frontier rows deferred to bfs_long this level
    int32_t long_rows[kBfsLongRows];
};

// Newly reached nodes collect in a per-wave LDS buffer of kBfsBuf entries, which goes to the
// queue with one atomic on its tail when it cannot take another 64 (and when the wave ends).
constexpr int kBfsBuf = 512;

struct BfsBuffer {
    int32_t* buf;   // this wave's kBfsBuf entries in LDS
    int32_t count;  // entries held (wave-uniform)
};

__device__ __forceinline__ void bfs_flush(BfsBuffer& b, int lane, int32_t* __restrict__ order, BfsState* st) {
    if (b.count == 0) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&st->tail, static_cast<uint32_t>(b.count));
    base = __shfl(base, 0, kWave);
    for (int32_t i = lane; i < b.count; i += kWave) order[base + i] = b.buf[i];
    b.count = 0;
}

// Expands entries k0 + lane of the row (k0 wave-uniform, entries from `end` on ignored): a
// neighbour still unreached is claimed for the next level and buffered for the queue.
__device__ __forceinline__ void bfs_expand(int32_t k0, int32_t end, int lane, int32_t level,
                                           const int32_t* __restrict__ col, int32_t* __restrict__ dist,
                                           int32_t* __restrict__ order, BfsState* st, BfsBuffer& b) {
    const int32_t k = k0 + lane;
    int32_t w = 0;
    bool found = false;
    if (k < end) {
        w = col[k];
        found = dist[w] == -1 && atomicCAS(&dist[w], -1, level + 1) == -1;
    }
    const uint64_t m = __ballot(found);
    if (m == 0) return;
    if (b.count > kBfsBuf - kWave) bfs_flush(b, lane, order, st);
    if (found) b.buf[b.count + __popcll(m & ((1ull << lane) - 1))] = w;
    b.count += __popcll(m);
}

// One wave per frontier node, lanes over its neighbours; rows longer than kBfsLongRow go to
// bfs_long (up to kBfsLongRows of them), so a hub's row does not hold the level on one wave.
__global__ void bfs_level(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                          int32_t* __restrict__ dist, int32_t* __restrict__ order, BfsState* st) {
    if (st->done) return;
    const uint32_t lo = st->lo, hi = st->hi;
    const int32_t level = st->level;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
    __shared__ int32_t lds[kBlock / kWave][kBfsBuf];
    BfsBuffer b{lds[threadIdx.x / kWave], 0};
    for (int64_t i = lo + wave; i < hi; i += nw) {
        const int32_t u = order[i];
        const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
        if (end - beg > kBfsLongRow) {
            uint32_t slot = 0;
            if (lane == 0) {
                slot = atomicAdd(&st->nlong, 1u);
                if (slot < kBfsLongRows) st->long_rows[slot] = u;
            }
            if (__shfl(slot, 0, kWave) < kBfsLongRows) continue;
        }
        for (int32_t k0 = beg; k0 < end; k0 += kWave) bfs_expand(k0, end, lane, level, col, dist, order, st, b);
    }
    bfs_flush(b, lane, order, st);
}

// The level's long rows, every wave taking every nw-th 64-entry chunk of each.
__global__ void bfs_long(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         int32_t* __restrict__ dist, int32_t* __restrict__ order, BfsState* st) {
    if (st->done) return;
    const uint32_t nl = st->nlong < kBfsLongRows ? st->nlong : kBfsLongRows;
    const int32_t level = st->level;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
    __shared__ int32_t lds[kBlock / kWave][kBfsBuf];
    BfsBuffer b{lds[threadIdx.x / kWave], 0};
    for (uint32_t j = 0; j < nl; ++j) {
        const int32_t u = st->long_rows[j];
        const int32_t beg = row_ptr[u], end = row_ptr[u + 1];
        for (int64_t k0 = beg + wave * kWave; k0 < end; k0 += nw * kWave)
            bfs_expand(static_cast<int32_t>(k0), end, lane, level, col, dist, order, st, b);
    }
    bfs_flush(b, lane, order, st);
}

__global__ void bfs_advance(BfsState* st) {
    if (st->done) return;
    st->nlong = 0;
    const uint32_t t = st->tail;
    if (t == st->hi) {
        st->done = 1;
        return;
    }
    st->lo = st->hi;
    st->hi = t;
    st->level += 1;
    st->depth = st->level;
}

__global__ void bfs_init(int32_t n, int32_t pivot, int32_t* __restrict__ dist, int32_t* __restrict__ order,
                         BfsState* st) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dist[u] = (u == pivot) ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        order[0] = pivot;
        st->tail = 1u;
        st->lo = 0u;
        st->hi = 1u;
        st->level = 0;
        st->done = 0;
        st->depth = 0;
        st->nlong = 0u;
    }
}

// Union-find with parent[x] <= x: find walks down to a root with path halving.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
    int32_t p = parent[x];
    while (p != x) {
        const int32_t gp = parent[p];
        if (gp != p) parent[x] = gp;   // halving; any value written is an ancestor of x
        x = p;
        p = gp;
    }
    return x;
}

__global__ void uf_init(int32_t n, int32_t* parent) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        parent[u] = static_cast<int32_t>(u);
}

__global__ void uf_hook(int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int32_t* parent) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int32_t ra = uf_find(parent, src[e]);
        int32_t rb = uf_find(parent, dst[e]);
        // max(ra, rb) strictly decreases on every failed attempt, so this terminates.
        while (ra != rb) {
            const int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
            const int32_t old = atomicCAS(&parent[hi], hi, lo);
            if (old == hi) break;
            ra = uf_find(parent, old);
            rb = uf_find(parent, lo);
        }
    }
}

// component[u] = the smallest input id of u's component (the union-find root).
__global__ void uf_flatten(int32_t n, int32_t* parent, int32_t* __restrict__ component) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        component[u] = uf_find(parent, static_cast<int32_t>(u));
}

// The nodes a breadth-first search from the pivot did not reach (other components), appended
// to its order in internal order: flags, their exclusive scan, then the scatter.
__global__ void unreached_flags(int32_t n, const int32_t* __restrict__ dist, uint32_t* __restrict__ flags) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u <= n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        flags[u] = (u < n && dist[u] < 0) ? 1u : 0u;
}

__global__ void append_unreached(int32_t n, uint32_t tail, const int32_t* __restrict__ dist,
                                 const uint32_t* __restrict__ pos, int32_t* __restrict__ order) {
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (dist[u] < 0) order[tail + pos[u]] = static_cast<int32_t>(u);
}

__global__ void uf_count_roots(int32_t n, const int32_t* __restrict__ parent, BuildScalars* sc) {
    int32_t c = 0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        c += (parent[u] == u);
    c = wave_sum(c);
    if ((threadIdx.x & (kWave - 1)) == 0 && c) atomicAdd(&sc->nroots, c);
}

int key_bits(int32_t n) {
    int b = 1;
    while (b < 31 && (static_cast<int64_t>(1) << b) < n) ++b;
    return b;
}

struct BuildLayout {
    int32_t* row_ptr;
    int32_t* col;
    float* weight;
    int32_t* edge_id;
    uint64_t* cdf;
    double* strength;
    uint32_t* rec;
    int32_t* bfs_order;
    int32_t* node_id;
    int32_t* node_index;
    int32_t* component;
    uint64_t* sfix;
    BuildScalars* scalars;
    size_t persistent;
    // scratch
    uint32_t* deg_in;
    uint64_t* sfix_in;
    uint64_t* keys_a;
    uint64_t* keys_b;
    int32_t* vals_a;
    int32_t* vals_b;
    uint32_t* hist;
    uint32_t* sums;
    int32_t* parent;
    BfsState* bfs;
    size_t total;
};

BuildLayout carve_build(void* ws, int32_t n, int64_t m, bool weighted) {
    Carver c(ws);
    BuildLayout L{};
    const int64_t nnz = 2 * m;
    L.row_ptr = c.take<int32_t>(n + 1);
    L.col = c.take<int32_t>(nnz);
    L.weight = c.take<float>(nnz);
    L.edge_id = c.take<int32_t>(nnz);
    L.cdf = weighted ? c.take<uint64_t>(nnz) : nullptr;
    L.strength = c.take<double>(n);
    L.rec = c.take<uint32_t>(static_cast<size_t>(kRecWords) * n);
    L.bfs_order = c.take<int32_t>(n);
    L.node_id = c.take<int32_t>(n);
    L.node_index = c.take<int32_t>(n);
    L.component = c.take<int32_t>(n);
    L.sfix = c.take<uint64_t>(n);
    L.scalars = c.take<BuildScalars>(1);
    L.persistent = c.used();
    // the sorts run over the 2m entries and over the n nodes
    const int64_t len = nnz > n ? nnz : n;
    L.deg_in = c.take<uint32_t>(n + 1);
    L.sfix_in = c.take<uint64_t>(n);
    L.keys_a = c.take<uint64_t>(len);
    L.keys_b = c.take<uint64_t>(len);
    L.vals_a = c.take<int32_t>(len);
    L.vals_b = c.take<int32_t>(len);
    const int64_t nb = blocks_for(len, kTile);
    L.hist = c.take<uint32_t>(256 * nb);
    const int64_t scan_len = (256 * nb > n + 1) ? 256 * nb : n + 1;
    L.sums = c.take<uint32_t>(blocks_for(scan_len, kTile) + 1);
    L.parent = c.take<int32_t>(n);
    L.bfs = c.take<BfsState>(1);
    L.total = c.used();
    return L;
}

int check_sizes(int32_t n, int64_t m) {
    if (n < 2) return fail(RWC_ERR_INVALID_ARG, "n = %d: a graph needs at least two nodes", n);
    if (m < 1) return fail(RWC_ERR_INVALID_ARG, "m = %lld: a graph needs at least one edge", (long long)m);
    if (n >= 0x7FFFFFFF) return fail(RWC_ERR_TOO_LARGE, "n = %d is too large", n);
    if (2 * m >= 0x7FFFFFFFll) return fail(RWC_ERR_TOO_LARGE, "2m = %lld entries exceed int32 offsets", (long long)(2 * m));
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_build_csr_workspace(int32_t n, int64_t m, int32_t weighted, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(check_sizes(n, m));
    *bytes = carve_build(nullptr, n, m, weighted != 0).total;
    return RWC_OK;
}

extern "C" int rwc_csr_persistent_bytes(int32_t n, int64_t m, int32_t weighted, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(check_sizes(n, m));
    *bytes = carve_build(nullptr, n, m, weighted != 0).persistent;
    return RWC_OK;
}

extern "C" int rwc_build_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const float* w,
                             void* ws, size_t ws_bytes, rwc_csr* out, void* stream) {
    return rwc_build_csr_ex(n, m, src, dst, w, 0u, ws, ws_bytes, out, stream);
}

extern "C" int rwc_build_csr_ex(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const float* w,
                                uint32_t flags, void* ws, size_t ws_bytes, rwc_csr* out, void* stream) {
    clear_error();
    if (!src || !dst || !out) return fail(RWC_ERR_INVALID_ARG, "src, dst and out must not be null");
    if (flags & ~static_cast<uint32_t>(RWC_BUILD_ALLOW_DISCONNECTED))
        return fail(RWC_ERR_INVALID_ARG, "unknown build flags 0x%x", flags);
    const bool allow_disconnected = (flags & RWC_BUILD_ALLOW_DISCONNECTED) != 0;
    RWC_CHECK(check_sizes(n, m));
    const bool weighted = (w != nullptr);
    const size_t need = carve_build(nullptr, n, m, weighted).total;
    RWC_CHECK(check_workspace(ws, ws_bytes, need));
    hipStream_t s = static_cast<hipStream_t>(stream);
    BuildLayout L = carve_build(ws, n, m, weighted);
    const int64_t nnz = 2 * m;
    const unsigned gs = 4096;  // grid-stride launches

    hipLaunchKernelGGL(init_scalars, dim3(1), dim3(1), 0, s, L.scalars);
    hipLaunchKernelGGL(validate_edges, dim3(blocks_for(m, kBlock) < gs ? blocks_for(m, kBlock) : gs), dim3(kBlock),
                       0, s, m, src, dst, w, n, L.scalars);
    RWC_HIP(hipGetLastError());
    BuildScalars host{};
    RWC_HIP(hipMemcpyAsync(&host, L.scalars, sizeof(host), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    RWC_CHECK(device_error_to_status(host.status));

    // degrees and weighted degrees by input id, then the internal order (see the top of the file)
    const unsigned gm = blocks_for(m, kBlock) < gs ? blocks_for(m, kBlock) : gs;
    const unsigned gn = blocks_for(n, kBlock) < gs ? blocks_for(n, kBlock) : gs;
    hipLaunchKernelGGL(fill_u32, dim3(blocks_for(n + 1, kBlock) < gs ? blocks_for(n + 1, kBlock) : gs), dim3(kBlock),
                       0, s, L.deg_in, static_cast<int64_t>(n) + 1, 0u);
    hipLaunchKernelGGL(fill_u32, dim3(blocks_for(2 * static_cast<int64_t>(n), kBlock) < gs
                                          ? blocks_for(2 * static_cast<int64_t>(n), kBlock)
                                          : gs),
                       dim3(kBlock), 0, s, reinterpret_cast<uint32_t*>(L.sfix_in), 2 * static_cast<int64_t>(n), 0u);
    hipLaunchKernelGGL(count_degrees, dim3(gm), dim3(kBlock), 0, s, m, src, dst, n, L.deg_in);
    if (weighted) hipLaunchKernelGGL(strength_in, dim3(gm), dim3(kBlock), 0, s, m, src, dst, w, L.sfix_in);
    hipLaunchKernelGGL(degree_stats, dim3(gn), dim3(kBlock), 0, s, n, L.deg_in, L.sfix_in, weighted, L.scalars);
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipMemcpyAsync(&host, L.scalars, sizeof(host), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    const bool by_strength = static_cast<int64_t>(host.max_deg_in) * n > 8 * m;   // max degree > 4 x mean
    if (by_strength) {
        int sbits = 1;
        while (sbits < 64 && (host.max_s_in >> sbits) != 0) ++sbits;
        hipLaunchKernelGGL(order_keys, dim3(gn), dim3(kBlock), 0, s, n, L.sfix_in, L.scalars, L.keys_a, L.vals_a);
        const int nbn = static_cast<int>(blocks_for(n, kTile));
        uint64_t *kin = L.keys_a, *kout = L.keys_b;
        int32_t *vin = L.vals_a, *vout = L.vals_b;
        for (int sh = 0; sh < sbits; sh += 8) {
            hipLaunchKernelGGL(radix_hist, dim3(nbn), dim3(kBlock), 0, s, kin, static_cast<int64_t>(n), sh, L.hist, nbn);
            RWC_CHECK(exclusive_scan(L.hist, L.hist, 256ll * nbn, L.sums, s));
            hipLaunchKernelGGL(radix_scatter, dim3(nbn), dim3(kBlock), 0, s, kin, vin, kout, vout,
                               static_cast<int64_t>(n), sh, L.hist, nbn);
            RWC_HIP(hipGetLastError());
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        RWC_HIP(hipMemcpyAsync(L.node_id, vin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(identity_order, dim3(gn), dim3(kBlock), 0, s, n, L.node_id);
    }
    // degrees in internal order -> row_ptr (exclusive scan over n + 1 counters, the last zero)
    uint32_t* deg = reinterpret_cast<uint32_t*>(L.row_ptr);
    hipLaunchKernelGGL(fill_u32, dim3(blocks_for(n + 1, kBlock) < gs ? blocks_for(n + 1, kBlock) : gs), dim3(kBlock),
                       0, s, deg, static_cast<int64_t>(n) + 1, 0u);
    hipLaunchKernelGGL(invert_order, dim3(gn), dim3(kBlock), 0, s, n, L.node_id, L.node_index, L.deg_in, deg);
    RWC_HIP(hipGetLastError());
    RWC_CHECK(exclusive_scan(deg, deg, static_cast<int64_t>(n) + 1, L.sums, s));

    // radix sort of directed entries by (internal row, input id of the neighbour)
    hipLaunchKernelGGL(make_keys, dim3(gm), dim3(kBlock), 0, s, m, src, dst, L.node_index, L.keys_a, L.vals_a);
    RWC_HIP(hipGetLastError());
    const int bits = key_bits(n);
    const int nb = static_cast<int>(blocks_for(nnz, kTile));
    uint64_t *kin = L.keys_a, *kout = L.keys_b;
    int32_t *vin = L.vals_a, *vout = L.vals_b;
    for (int field = 0; field < 2; ++field) {
        for (int sh = 0; sh < bits; sh += 8) {
            const int shift = field * 32 + sh;
            hipLaunchKernelGGL(radix_hist, dim3(nb), dim3(kBlock), 0, s, kin, nnz, shift, L.hist, nb);
            RWC_CHECK(exclusive_scan(L.hist, L.hist, 256ll * nb, L.sums, s));
            hipLaunchKernelGGL(radix_scatter, dim3(nb), dim3(kBlock), 0, s, kin, vin, kout, vout, nnz, shift, L.hist,
                               nb);
            RWC_HIP(hipGetLastError());
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
    }
    hipLaunchKernelGGL(fill_csr, dim3(blocks_for(nnz, kBlock) < gs ? blocks_for(nnz, kBlock) : gs), dim3(kBlock), 0,
                       s, nnz, kin, vin, w, L.node_index, L.col, L.edge_id, L.weight, L.scalars);
    hipLaunchKernelGGL(row_pass, dim3(blocks_for(static_cast<int64_t>(n) * kWave, kBlock) < gs
                                          ? blocks_for(static_cast<int64_t>(n) * kWave, kBlock)
                                          : gs),
                       dim3(kBlock), 0, s, n, L.row_ptr, L.weight, L.cdf, L.strength, L.sfix, L.scalars);
    hipLaunchKernelGGL(build_records, dim3(gn), dim3(kBlock), 0, s, n, L.row_ptr, L.col, L.cdf, L.node_id, L.rec);
    hipLaunchKernelGGL(pick_pivot, dim3(gn), dim3(kBlock), 0, s, n, L.sfix, L.scalars);
    hipLaunchKernelGGL(pivot_input_id, dim3(1), dim3(1), 0, s, L.node_id, L.scalars);
    hipLaunchKernelGGL(uf_init, dim3(blocks_for(n, kBlock) < gs ? blocks_for(n, kBlock) : gs), dim3(kBlock), 0, s, n,
                       L.parent);
    hipLaunchKernelGGL(uf_hook, dim3(blocks_for(m, kBlock) < gs ? blocks_for(m, kBlock) : gs), dim3(kBlock), 0, s, m,
                       src, dst, L.parent);
    hipLaunchKernelGGL(uf_count_roots, dim3(blocks_for(n, kBlock) < gs ? blocks_for(n, kBlock) : gs), dim3(kBlock), 0,
                       s, n, L.parent, L.scalars);
    // component ids by input id, before the breadth-first search takes over the union-find scratch
    hipLaunchKernelGGL(uf_flatten, dim3(gn), dim3(kBlock), 0, s, n, L.parent, L.component);
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipMemcpyAsync(&host, L.scalars, sizeof(host), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    RWC_CHECK(device_error_to_status(host.status));
    if (host.nroots != 1 && !allow_disconnected)
        return fail(RWC_ERR_DISCONNECTED, "the graph has %d connected components", host.nroots);

    // breadth-first start order from the pivot (the union-find scratch holds the distances):
    // levels are launched kBfsChunk at a time and the host looks once per chunk (a deep mesh's
    // hundreds of levels cost a few round trips, not one each); levels past the last return
    // at once
    hipLaunchKernelGGL(bfs_init, dim3(blocks_for(n, kBlock) < gs ? blocks_for(n, kBlock) : gs), dim3(kBlock), 0, s, n,
                       host.pivot, L.parent, L.bfs_order, L.bfs);
    RWC_HIP(hipGetLastError());
    constexpr int kBfsChunk = 32;
    BfsState bs{};
    for (int32_t launched = 0; !bs.done; launched += kBfsChunk) {
        if (launched > n) return fail(RWC_ERR_HIP, "breadth-first search did not finish in %d levels", n);
        for (int c = 0; c < kBfsChunk; ++c) {
            hipLaunchKernelGGL(bfs_level, dim3(gs), dim3(kBlock), 0, s, L.row_ptr, L.col, L.parent, L.bfs_order, L.bfs);
            hipLaunchKernelGGL(bfs_long, dim3(gs), dim3(kBlock), 0, s, L.row_ptr, L.col, L.parent, L.bfs_order, L.bfs);
            hipLaunchKernelGGL(bfs_advance, dim3(1), dim3(1), 0, s, L.bfs);
        }
        RWC_HIP(hipGetLastError());
        RWC_HIP(hipMemcpyAsync(&bs, L.bfs, sizeof(bs), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
    }
    if (bs.tail != static_cast<uint32_t>(n)) {
        if (host.nroots == 1 || !allow_disconnected)
            return fail(RWC_ERR_DISCONNECTED, "breadth-first search stopped at %u of %d nodes", bs.tail, n);
        // the other components' nodes follow the pivot's component, in internal order
        uint32_t* pos = reinterpret_cast<uint32_t*>(L.keys_b);   // n + 1 counters; the sort is done
        hipLaunchKernelGGL(unreached_flags, dim3(blocks_for(n + 1, kBlock) < gs ? blocks_for(n + 1, kBlock) : gs),
                           dim3(kBlock), 0, s, n, L.parent, pos);
        RWC_CHECK(exclusive_scan(pos, pos, static_cast<int64_t>(n) + 1, L.sums, s));
        hipLaunchKernelGGL(append_unreached, dim3(gn), dim3(kBlock), 0, s, n, bs.tail, L.parent, pos, L.bfs_order);
        RWC_HIP(hipGetLastError());
    }
    const int32_t depth = bs.depth;

    rwc_csr g{};
    g.n = n;
    g.pivot = host.pivot_id;
    g.m = m;
    g.nnz = nnz;
    g.weighted = weighted ? 1 : 0;
    g.max_degree = host.max_deg;
    g.vol_fixed = host.vol_fixed;
    g.vol = static_cast<double>(host.vol_fixed) * (1.0 / 16777216.0);
    g.row_ptr = L.row_ptr;
    g.col = L.col;
    g.weight = L.weight;
    g.edge_id = L.edge_id;
    g.cdf = L.cdf;
    g.strength = L.strength;
    g.rec = L.rec;
    g.bfs_order = L.bfs_order;
    g.bfs_depth = depth;
    g.node_id = L.node_id;
    g.node_index = L.node_index;
    g.pivot_index = host.pivot;
    g.internal_order = by_strength ? 1 : 0;
    g.components = host.nroots;
    g.component = L.component;
    *out = g;
    return RWC_OK;
}
