// Device-side building blocks of the sampler: the counter-based generator, neighbour
// selection, the per-(tree, node) state word and wave-level reductions.  gfx950, wave64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rwc {

constexpr int kWave = 64;

// Pointers the hot loops dereference, retagged as global memory: loaded from argument
// structs they are generic, which makes every access a flat instruction (64-bit addresses,
// and counted with LDS traffic so that waits for LDS also wait for HBM).
#define RWC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RWC_GLOBAL T* global_ptr(T* p) {
    return (RWC_GLOBAL T*)p;
}
#define RWC_LDS __attribute__((address_space(3)))
// Waits until every vector memory operation of this wave has completed, including copies
// from memory into LDS, which the compiler does not track (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// 16-byte load through such a pointer (HIP's vector types only bind generic references)
__device__ __forceinline__ uint4 load_u4(const RWC_GLOBAL uint4* p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = *reinterpret_cast<const RWC_GLOBAL u32x4*>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64 products
// on counter words 0 and 2, key words added in each round and bumped by the Weyl
// constants between rounds.  Only output words 0 and 1 are used; the compiler drops the
// rest of the last round.
// ---------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t philox_x64(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;   // v_mul_lo/hi_u32 on the GPU
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
        const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return static_cast<uint64_t>(c0) | (static_cast<uint64_t>(c1) << 32);
}

// floor(a * b / 2^64)
__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// All four output words of Philox4x32-10 (same rounds as philox_x64).
__device__ __forceinline__ uint4 philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------------------
// Stratified stack entries: Latin hypercube sampling (McKay, Beckman, Conover 1979) of each
// stack entry over the samples 0 .. L-1 of a call.  Entry (u, k) of sample i takes stratum
// sigma(i) of [0, 2^64) split into L strata of width floor(2^64 / L), and its own Philox word
// x places it inside the stratum.  sigma is a permutation of 0 .. L-1 keyed by the entry
// through one Philox call a on (k, u, 2^32 - 1, g): a 4-round unbalanced Feistel network on
// B = max(2, ceil(log2 L)) bits (high part floor(B/2) bits, low part the rest; a round maps
// (high, low) to (low, high xor (fmix32(low xor key) mod 2^|high|)), the widths trading
// places; keys a0, a1, a0 xor rotl(a1, 16), a1 xor rotl(a0, 16); fmix32 is the MurmurHash3
// 32-bit finaliser), walked until it lands below L, then shifted by s = floor(b L / 2^64),
// b = a2 + 2^32 a3.  The shift makes sigma(i) uniform for every i, so one sample's entries
// stay independent and uniform and every tree is still a Wilson tree; over the L samples each
// entry takes every stratum once.  Needs i < L <= 2^31 (the key counter is never a sample's).
// ---------------------------------------------------------------------------------------
struct Strata {
    uint64_t width;   // floor(2^64 / L)
    uint32_t count;   // L; below 2 the draws are not stratified
    uint32_t bits;    // B: the Feistel network permutes [0, 2^B), 2^B >= L
};

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint64_t stratified_word(uint64_t x, uint32_t k, uint32_t u, uint32_t i, uint32_t g,
                                                    uint32_t k0, uint32_t k1, const Strata& S) {
    const uint4 a = philox4(k, u, 0xFFFFFFFFu, g, k0, k1);
    const uint32_t key2 = a.x ^ __builtin_rotateleft32(a.y, 16), key3 = a.y ^ __builtin_rotateleft32(a.x, 16);
    const uint32_t p = S.bits >> 1, q = S.bits - p;   // widths of the high and low parts
    const uint32_t mp = (1u << p) - 1u, mq = (1u << q) - 1u;
    // Cycle walking: i < L (the host checks every call's sample range) lies on its own cycle
    // of the permutation of [0, 2^B), so a value below L comes back; each step lands there
    // with probability above 1/2, so the cap is never reached in practice.  The clamp below
    // keeps even an out-of-range index inside the row.
    uint32_t y = i;
    uint32_t walks = 0;
    do {
        // rounds 1 and 3 see (p-bit high, q-bit low), rounds 2 and 4 (q-bit high, p-bit low)
        uint32_t hi = y >> q, lo = y & mq;
        uint32_t t = hi ^ (fmix32(lo ^ a.x) & mp);    // p bits
        hi = lo;                                      // q bits
        lo = t;
        t = hi ^ (fmix32(lo ^ a.y) & mq);             // q bits
        hi = lo;                                      // p bits
        lo = t;
        t = hi ^ (fmix32(lo ^ key2) & mp);
        hi = lo;
        lo = t;
        t = hi ^ (fmix32(lo ^ key3) & mq);
        hi = lo;
        lo = t;
        y = (hi << q) | lo;
    } while (y >= S.count && ++walks < (1u << 16));
    if (y >= S.count) y = 0;
    const uint64_t b = static_cast<uint64_t>(a.z) | (static_cast<uint64_t>(a.w) << 32);
    uint32_t sigma = y + static_cast<uint32_t>(mulhi64(b, S.count));   // both < L <= 2^31
    if (sigma >= S.count) sigma -= S.count;
    return static_cast<uint64_t>(sigma) * S.width + mulhi64(x, S.width);
}

// RandomNeighbor, unweighted: the position within the row of the chosen neighbour,
// floor(x * deg / 2^64).  (Weighted rows: the first position k with floor(x * S / 2^64) <
// cdf[beg + k], S = cdf[end - 1]; the search lives with the node records in the sampler.)
__device__ __forceinline__ int32_t select_unweighted(uint64_t x, int32_t deg) {
    return static_cast<int32_t>(mulhi64(x, static_cast<uint64_t>(deg)));
}

// Node records (rwc_csr::rec): 16 x uint32 per node (in the graph's internal order), 64-byte
// aligned.  Word 0 is the degree, word 1 the row offset and word 2 the node's input id (the
// id the generator is keyed on).  Unweighted rows store the internal indices of their first
// 13 neighbours in words 3..15 (position p in word 3 + p).  Weighted rows store those of their
// first 3 entries in words 3..5, the row's total (its last CDF value) in words 6..7 and the
// CDF values of the first 3 entries in words 8..13.  Whatever degree the row has, these
// positions need no read of the row itself.
constexpr int kRecWords = 16;
constexpr int kRecId = 2;               // word holding the node's input id
constexpr int kRecFirst = 3;            // word of the first inline neighbour
constexpr int kRecInline = 13;          // neighbours stored inline for unweighted rows
constexpr int kRecInlineWeighted = 3;   // (id, cdf) pairs stored inline for weighted rows

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014): the tree checksum term.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------------------
// Per-(tree, node) state word, 64 bits:
//   [31:0]  next  -- the last neighbour chosen at a departure (Next[u] of Algorithm 3);
//                    the parent once the node is in the tree
//   [55:32] cnt   -- departures from the node in this tree (the Philox step word)
//   [61:56] owner -- walker lane that holds the node on its current path (multi-walker)
//   [62]    OWNED -- the node is on a live walker path
//   [63]    INTREE
// The all-zero word is a fresh node; the root starts as INTREE.
// ---------------------------------------------------------------------------------------
constexpr uint64_t kInTree = 1ull << 63;
constexpr uint64_t kOwned = 1ull << 62;
constexpr uint32_t kCntMax = (1u << 24) - 1;

__device__ __forceinline__ uint32_t st_next(uint64_t w) { return static_cast<uint32_t>(w); }
__device__ __forceinline__ uint32_t st_cnt(uint64_t w) {
    return static_cast<uint32_t>(w >> 32) & 0xFFFFFFu;
}
__device__ __forceinline__ uint32_t st_owner(uint64_t w) {
    return static_cast<uint32_t>(w >> 56) & 0x3Fu;
}
__device__ __forceinline__ uint64_t st_make(uint32_t next, uint32_t cnt) {
    return static_cast<uint64_t>(next) | (static_cast<uint64_t>(cnt) << 32);
}
__device__ __forceinline__ uint64_t st_make_owned(uint32_t next, uint32_t cnt, uint32_t owner) {
    return st_make(next, cnt) | kOwned | (static_cast<uint64_t>(owner) << 56);
}

// Square of a departure count as uint64.  The count is known to fit 24 bits; the empty asm
// hides that from the optimiser, whose fold of a 24-bit multiply plus 64-bit add into
// v_mad_u64_u32 drops the 24-bit mask (seen with the ROCm 7.2 compiler for gfx950) and would
// square the raw word including the flag bits.  The asm holds no memory operation.
__device__ __forceinline__ uint64_t square_count(uint32_t c) {
    asm volatile("" : "+v"(c));
    return static_cast<uint64_t>(c) * c;
}

// ---------------------------------------------------------------------------------------
// Wave reductions (wave64, shuffles).
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace rwc
