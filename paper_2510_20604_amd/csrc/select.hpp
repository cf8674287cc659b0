// RandomNeighbor (Algorithm 3) on the 64-byte node records: the neighbour chosen at a node by
// 64 random bits, read from the record wherever it holds the answer.  Shared by the Wilson
// walk kernels and the trap-walk kernel.
#pragma once

#include "device.hpp"

namespace rwc {
namespace {

// Word i (0..15) of a node record held in four uint4 registers.
__device__ __forceinline__ uint32_t rec_word(const uint4& a, const uint4& b, const uint4& c, const uint4& d,
                                             uint32_t i) {
    const uint4 q = (i < 4) ? a : (i < 8) ? b : (i < 12) ? c : d;
    const uint32_t s = i & 3u;
    return s == 0 ? q.x : (s == 1 ? q.y : (s == 2 ? q.z : q.w));
}

// RandomNeighbor (Algorithm 3): the neighbour chosen at a node by the 64 random bits x (its
// internal index), read from the node's record wherever it holds the answer.  rec(i) returns
// word i of the record, already local (registers or LDS).  Rows list their neighbours by
// ascending input id.  Unweighted: position floor(x deg / 2^64), inline below kRecInline.
// Weighted: the first position k with floor(x S / 2^64) < cdf[k], S the row's total; the
// record's three CDF values settle it without a read of the row whenever r falls below the
// third, else a binary search over the rest of the row's CDF does.
template <class Rec>
__device__ __forceinline__ uint32_t choose_neighbor(uint64_t x, Rec rec, const RWC_GLOBAL int32_t* col,
                                                    const RWC_GLOBAL uint64_t* cdf) {
    const uint32_t deg = rec(0);
    const int32_t beg = static_cast<int32_t>(rec(1));
    uint32_t pos;
    if (cdf == nullptr) {
        pos = static_cast<uint32_t>(select_unweighted(x, static_cast<int32_t>(deg)));
        if (pos < static_cast<uint32_t>(kRecInline)) return rec(static_cast<uint32_t>(kRecFirst) + pos);
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
            return rec(static_cast<uint32_t>(kRecFirst) + pos);
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

}  // namespace
}  // namespace rwc
