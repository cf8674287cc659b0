// Status strings, per-thread error detail and device queries.
#include "common.hpp"

#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

namespace rwc {

namespace {
thread_local std::string g_last_error;
}

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

void clear_error() {
    g_last_error.clear();
    // drop an error state left by earlier HIP calls of other code in this thread, so that the
    // launch checks of this call report only its own failures
    (void)hipGetLastError();
}

int device_error_to_status(uint32_t bits) {
    if (bits == 0) return RWC_OK;
    if (bits & kErrNodeRange) return fail(RWC_ERR_NODE_RANGE, "a node id (edge endpoint or root) is outside [0, n)");
    if (bits & kErrSelfLoop) return fail(RWC_ERR_SELF_LOOP, "the edge list contains a self-loop");
    if (bits & kErrDupEdge) return fail(RWC_ERR_DUP_EDGE, "the edge list repeats an undirected edge");
    if (bits & kErrWeight)
        return fail(RWC_ERR_WEIGHT_RANGE, "an edge weight is not a float32 value in [0.5, 65536)");
    if (bits & kErrStrength)
        return fail(RWC_ERR_WEIGHT_RANGE, "a weighted degree reaches 2^53 (fixed-point overflow)");
    if (bits & kErrVolume)
        return fail(RWC_ERR_WEIGHT_RANGE, "the total weight times 2^24 reaches 2^64 (fixed-point overflow)");
    if (bits & kErrDupRoot) return fail(RWC_ERR_INVALID_ARG, "the root set lists a node twice");
    if (bits & kErrNonFinite) return fail(RWC_ERR_INVALID_ARG, "an input value is not finite");
    if (bits & kErrCapacity)
        return fail(RWC_ERR_TOO_LARGE, "the factor or inverse pool, or a column's sort buffer, is full");
    if (bits & kErrPivot) return fail(RWC_ERR_BREAKDOWN, "the incomplete factorization met a non-positive pivot");
    if (bits & kErrNotConverged)
        return fail(RWC_ERR_NOT_CONVERGED, "the solve missed its tolerance within max_iter iterations");
    if (bits & kErrStepLimit)
        return fail(RWC_ERR_STEP_LIMIT, "a tree exceeded max_steps_per_tree walk steps");
    if (bits & kErrCountOverflow)
        return fail(RWC_ERR_COUNT_OVERFLOW, "a node departed 2^24 times within one tree");
    if (bits & kErrProtocol)
        return fail(RWC_ERR_HIP, "multi-walker protocol invariant violated (device bits 0x%x)", bits);
    if (bits & kErrUncovered)
        return fail(RWC_ERR_DISCONNECTED, "the root set misses a connected component of the graph");
    if (bits & kErrWait)
        return fail(RWC_ERR_HIP, "a FastChol inverse column waited too long for a column it reads");
    if (bits & kErrRetrace)
        return fail(RWC_ERR_STEP_LIMIT, "loop-erased path retrace exceeded n nodes");
    return fail(RWC_ERR_HIP, "unknown device error bits 0x%x", bits);
}

int device_cu_count() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (static_cast<int>(cache.size()) <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

}  // namespace rwc

extern "C" const char* rwc_status_string(int status) {
    switch (status) {
        case RWC_OK: return "ok";
        case RWC_ERR_INVALID_ARG: return "invalid argument";
        case RWC_ERR_NODE_RANGE: return "edge endpoint out of range";
        case RWC_ERR_SELF_LOOP: return "self-loop";
        case RWC_ERR_DUP_EDGE: return "duplicate edge";
        case RWC_ERR_WEIGHT_RANGE: return "weight out of range";
        case RWC_ERR_DISCONNECTED: return "graph is not connected";
        case RWC_ERR_TOO_LARGE: return "graph too large";
        case RWC_ERR_WORKSPACE: return "workspace too small or misaligned";
        case RWC_ERR_STEP_LIMIT: return "walk step limit exceeded";
        case RWC_ERR_COUNT_OVERFLOW: return "per-tree departure count overflow";
        case RWC_ERR_NOT_CONVERGED: return "solver did not converge";
        case RWC_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

extern "C" int rwc_last_error(char* buf, size_t len) {
    const std::string& s = rwc::g_last_error;
    if (buf && len) {
        size_t k = s.size() < len - 1 ? s.size() : len - 1;
        std::memcpy(buf, s.data(), k);
        buf[k] = '\0';
    }
    return static_cast<int>(s.size());
}

extern "C" int rwc_workspace_status(const void* ws, void* stream) {
    using namespace rwc;
    clear_error();
    if (!ws) return fail(RWC_ERR_INVALID_ARG, "workspace is null");
    WsHeader h{};
    hipStream_t s = static_cast<hipStream_t>(stream);
    RWC_HIP(hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    if (h.tag != kHeaderTag) return fail(RWC_ERR_INVALID_ARG, "the workspace holds no call's status");
    return device_error_to_status(h.status);
}

extern "C" int rwc_workspace_iterations(const void* ws, int32_t* iters, void* stream) {
    using namespace rwc;
    clear_error();
    if (!ws || !iters) return fail(RWC_ERR_INVALID_ARG, "workspace and iters are required");
    WsHeader h{};
    hipStream_t s = static_cast<hipStream_t>(stream);
    RWC_HIP(hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    if (h.tag != kHeaderTag) return fail(RWC_ERR_INVALID_ARG, "the workspace holds no call's status");
    *iters = h.iters;
    return RWC_OK;
}
