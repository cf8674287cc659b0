// Host-side helpers shared by the library's translation units: error reporting, workspace
// carving and launch-shape arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "rwc.h"

namespace rwc {

// Records a detail message for rwc_last_error() on the calling thread and returns `status`.
int fail(int status, const char* fmt, ...);
void clear_error();

#define RWC_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::rwc::fail(RWC_ERR_HIP, "%s failed: %s (%s:%d)", #call,                \
                               hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

#define RWC_CHECK(status)                                                                  \
    do {                                                                                   \
        int s_ = (status);                                                                 \
        if (s_ != RWC_OK) return s_;                                                       \
    } while (0)

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Sequential carving of a caller-owned workspace into 256-byte aligned regions.  With a
// null base it only measures.
class Carver {
  public:
    explicit Carver(void* base = nullptr) : base_(static_cast<char*>(base)) {}
    template <typename T>
    T* take(size_t count) {
        size_t off = off_;
        off_ = align_up(off_ + count * sizeof(T));
        return base_ ? reinterpret_cast<T*>(base_ + off) : nullptr;
    }
    size_t used() const { return off_; }

  private:
    char* base_;
    size_t off_ = 0;
};

// Calls whose walks or solves end at one node need a connected graph.
inline int require_connected(const rwc_csr* g, const char* what) {
    if (g && g->components > 1)
        return fail(RWC_ERR_DISCONNECTED, "%s needs a connected graph (this CSR has %d components)", what,
                    g->components);
    return RWC_OK;
}

inline int check_workspace(const void* ws, size_t have, size_t need) {
    if (need > 0 && ws == nullptr) return fail(RWC_ERR_WORKSPACE, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
        return fail(RWC_ERR_WORKSPACE, "workspace is not %zu-byte aligned", kAlign);
    if (have < need)
        return fail(RWC_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
    return RWC_OK;
}

inline unsigned blocks_for(int64_t work, int per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    return static_cast<unsigned>(b < 1 ? 1 : b);
}

// Device-side error bits written with atomicOr into a status word; translated on the host.
enum DeviceError : uint32_t {
    kErrNodeRange = 1u << 0,
    kErrSelfLoop = 1u << 1,
    kErrDupEdge = 1u << 2,
    kErrWeight = 1u << 3,
    kErrStepLimit = 1u << 4,
    kErrCountOverflow = 1u << 5,
    kErrStrength = 1u << 6,
    kErrRetrace = 1u << 7,
    kErrProtocol = 1u << 8,
    kErrVolume = 1u << 9,
    kErrNotConverged = 1u << 10,
    kErrDupRoot = 1u << 11,
    kErrNonFinite = 1u << 12,
    kErrCapacity = 1u << 13,    // a FastChol pool or a column's sort buffer is full
    kErrPivot = 1u << 14,       // a non-positive pivot in the incomplete factorization
    kErrUncovered = 1u << 16,   // a root set misses a connected component
    kErrWait = 1u << 15,        // a FastChol inverse column outwaited its spin limit
};

int device_error_to_status(uint32_t bits);

// The first kHeaderBytes of every sampling, estimate and adjoint workspace.  The first kernel
// of each call sets `tag` and clears `status`; later kernels of the call OR error bits
// (DeviceError) into `status`, so the outcome of a call that returned before its device work
// finished can be read afterwards (rwc_workspace_status).
struct WsHeader {
    uint32_t status;
    uint32_t tag;
    int32_t iters;      // solve iterations run (estimate)
    uint32_t reserved;
};
constexpr size_t kHeaderBytes = 256;
constexpr uint32_t kHeaderTag = 0x52574331u;

__device__ __forceinline__ void header_begin(WsHeader* h) {
    h->status = 0;
    h->tag = kHeaderTag;
    h->iters = 0;
}

// Number of compute units of the current device (cached per device).
int device_cu_count();
// Waves of the walker-team kernel (with or without the LDS path ring) resident on the whole
// device at once (occupancy x compute units); defined with the kernels.
int team_resident_waves(bool ring);

}  // namespace rwc
