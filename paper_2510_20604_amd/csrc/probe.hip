// Measurement kernels of rwc_probe.h: a dependent random-gather chain kernel (the access
// pattern of a walker) and a streaming copy.
#include "rwc_probe.h"

#include "common.hpp"
#include "device.hpp"

namespace rwc {
namespace {

__global__ void __launch_bounds__(256) gather_chains(const uint64_t* __restrict__ table, uint64_t words,
                                                     int64_t lanes, int32_t chain_len, uint32_t seed,
                                                     uint64_t* __restrict__ sink) {
    const int64_t lane = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (lane >= lanes) return;
    uint64_t x = splitmix64(static_cast<uint64_t>(lane) ^ (static_cast<uint64_t>(seed) << 40));
    uint64_t acc = 0;
    for (int32_t i = 0; i < chain_len; ++i) {
        const uint64_t v = table[mulhi64(x, words)];
        acc += v;
        x = splitmix64(x + v);
    }
    // practically never taken; keeps every load live
    if (acc == 0x5A5A5A5A5A5A5A5Aull) sink[lane] = acc;
}

__global__ void __launch_bounds__(256) copy_words(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                  uint64_t words) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < words; i += stride)
        dst[i] = src[i];
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {   // teardown: failures here have nobody to report to
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_probe_random_gather(const uint64_t* table, uint64_t words, int64_t lanes, int32_t chain_len,
                                       uint32_t seed, uint64_t* sink, float* ms_out, void* stream) {
    clear_error();
    if (!table || !sink || !ms_out || words == 0 || lanes <= 0 || chain_len <= 0)
        return fail(RWC_ERR_INVALID_ARG, "bad probe arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    EventPair ev;
    RWC_HIP(hipEventCreate(&ev.a));
    RWC_HIP(hipEventCreate(&ev.b));
    RWC_HIP(hipEventRecord(ev.a, s));
    hipLaunchKernelGGL(gather_chains, dim3(blocks_for(lanes, 256)), dim3(256), 0, s, table, words, lanes, chain_len,
                       seed, sink);
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipEventRecord(ev.b, s));
    RWC_HIP(hipEventSynchronize(ev.b));
    RWC_HIP(hipEventElapsedTime(ms_out, ev.a, ev.b));
    return RWC_OK;
}

extern "C" int rwc_probe_copy(const uint64_t* src, uint64_t* dst, uint64_t words, float* ms_out, void* stream) {
    clear_error();
    if (!src || !dst || !ms_out || words == 0) return fail(RWC_ERR_INVALID_ARG, "bad probe arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    EventPair ev;
    RWC_HIP(hipEventCreate(&ev.a));
    RWC_HIP(hipEventCreate(&ev.b));
    const unsigned grid = 256u * 16u;
    RWC_HIP(hipEventRecord(ev.a, s));
    hipLaunchKernelGGL(copy_words, dim3(grid), dim3(256), 0, s, src, dst, words);
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipEventRecord(ev.b, s));
    RWC_HIP(hipEventSynchronize(ev.b));
    RWC_HIP(hipEventElapsedTime(ms_out, ev.a, ev.b));
    return RWC_OK;
}
