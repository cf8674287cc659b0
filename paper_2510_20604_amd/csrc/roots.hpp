// Root sets on graphs of several connected components (RWC_BUILD_ALLOW_DISCONNECTED): every
// component needs a root, or its walks would never end and its grounded system would be
// singular.  cover[c] marks the components that hold a root (c is the component's smallest
// input id, the CSR's `component` entry); a node of an unmarked component is reported and, so
// that whatever the call has enqueued after the check still ends, added to the root mask (one
// bit per internal index) as if it were a root.  The caller discards such a call's outputs.
#pragma once

#include "common.hpp"

namespace rwc {
namespace {

__global__ void cover_clear(int32_t n, uint32_t* __restrict__ cover) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        cover[i] = 0u;
}

// Root ids out of range are left to the mask kernels, which report them.
__global__ void cover_mark(const int32_t* __restrict__ roots, int32_t nroots, int32_t n,
                           const int32_t* __restrict__ component, uint32_t* __restrict__ cover) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nroots) return;
    const int32_t id = roots[i];
    if (id >= 0 && id < n) cover[component[id]] = 1u;
}

__global__ void cover_check(int32_t n, const int32_t* __restrict__ component, const int32_t* __restrict__ node_index,
                            const uint32_t* __restrict__ cover, uint32_t* __restrict__ mask, WsHeader* header) {
    bool missed = false;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (cover[component[u]] == 0u) {
            missed = true;
            const int32_t x = node_index[u];
            atomicOr(&mask[x >> 5], 1u << (x & 31));
        }
    }
    if (missed) atomicOr(&header->status, static_cast<uint32_t>(kErrUncovered));
}

// The three launches, after the root mask has been built.
inline void check_root_cover(const rwc_csr& g, const int32_t* roots, int32_t nroots, uint32_t* cover, uint32_t* mask,
                             WsHeader* header, hipStream_t s) {
    const unsigned nb = blocks_for(g.n, 256) < 4096 ? blocks_for(g.n, 256) : 4096;
    hipLaunchKernelGGL(cover_clear, dim3(nb), dim3(256), 0, s, g.n, cover);
    hipLaunchKernelGGL(cover_mark, dim3(blocks_for(nroots, 256)), dim3(256), 0, s, roots, nroots, g.n, g.component,
                       cover);
    hipLaunchKernelGGL(cover_check, dim3(nb), dim3(256), 0, s, g.n, g.component, g.node_index, cover, mask, header);
}

}  // namespace
}  // namespace rwc
