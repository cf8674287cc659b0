// rwc_estimate: the pivot solve and the assembly of AppRWC (Algorithm 1) for the FastWalk
// estimate of Algorithm 3.
//
// The pivot column of calL^+ that Algorithm 1 obtains from one Laplacian solve is expressed
// through the hitting times to the pivot v: h_u = H_uv solves L_v h = d_{-v} (the first-step
// equations multiplied by D, grounded at v), and (calL^+)_uv = sqrt(d_u d_v)(RWC_v - h_u)/vol.
// Substituting into Eq. (3) with (calL_v^{-1})_uu estimated by t~_u = C_u / l gives
//     RWC_u = vol t~_u / d_u - 2 h_u + RWC_v,   RWC_v = sum_u d_u h_u / vol.
// L_v is symmetric positive definite, so the solve is Jacobi-preconditioned conjugate
// gradients in FP64.  Dot products use fixed per-block partials summed in a fixed order, so
// results are bitwise reproducible run to run.  This file is compiled without FMA
// contraction.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "roots.hpp"
#include "device.hpp"

namespace rwc {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

struct Scalars {
    double rz;      // r^T z of the current iterate
    double alpha;
    double beta;
    double rr;      // r^T r
    double rr0;     // ||b||^2
    double rwc_v;   // RWC of the pivot (of the root set for the group estimate)
    int32_t done;   // the residual met the tolerance: later iteration kernels return at once
    int32_t iters;  // iterations completed
};

// Grounded nodes: the pivot v, or the root set of the group estimate (bitmap of n bits).
__device__ __forceinline__ bool grounded(const uint32_t* __restrict__ gmask, int32_t v, int64_t u) {
    return gmask ? ((gmask[u >> 5] >> (u & 31)) & 1u) != 0 : u == v;
}

__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / kWave; ++w) s += lds[w];
    __syncthreads();
    return s;  // valid in thread 0
}

__global__ void pcg_init(int32_t n, int32_t v, const uint32_t* __restrict__ gmask, const double* __restrict__ d,
                         double* __restrict__ x, double* __restrict__ r, double* __restrict__ z, double* __restrict__ p,
                         double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double rz = 0.0, rr = 0.0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool gu = grounded(gmask, v, u);
        const double ru = gu ? 0.0 : d[u];
        const double zu = gu ? 0.0 : ru / d[u];
        x[u] = 0.0;
        r[u] = ru;
        z[u] = zu;
        p[u] = zu;
        rz += ru * zu;
        rr += ru * ru;
    }
    rz = block_sum(rz, lds);
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rz;
        part[2 * blockIdx.x + 1] = rr;
    }
}

// y = L_v p on the grounded system (row and column v removed, p_v kept at zero).  Block b owns
// rows b, b + nb, b + 2 nb, ... (nb blocks), so hub rows, which cluster at small ids in
// power-law graphs, land in different blocks.  kRowLanes lanes share a short row (strided over its
// entries, then a shuffle reduction); rows longer than kLongRow are left out of that pass and
// then taken one at a time, in order, by the whole block.
constexpr int kRowLanes = 16;
constexpr int kLongRow = 16 * kRowLanes;

__global__ void spmv_dot(int32_t n, int32_t v, const uint32_t* __restrict__ gmask, const Scalars* __restrict__ sc,
                         const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const float* __restrict__ weight, const double* __restrict__ d, const double* __restrict__ p,
                         double* __restrict__ ap, double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    __shared__ uint64_t long_mask[kBlock / kWave];
    if (sc->done) return;
    const int sub = threadIdx.x & (kRowLanes - 1);
    const int group = threadIdx.x / kRowLanes;
    constexpr int kGroups = kBlock / kRowLanes;
    const int64_t b = blockIdx.x, nb = gridDim.x;
    double acc = 0.0;
    // A row's loads form a chain (bounds, entries, gathers).  The next row's bounds and this
    // row's d and p are loaded before this row's entries, and a lane loads four entries, then
    // their four gathers, before it adds them (in entry order), so fewer latencies follow one
    // another.
    const int64_t ustep = static_cast<int64_t>(kGroups) * nb;
    int64_t u = b + group * nb;
    int32_t beg = 0, end = 0;
    if (u < n) {
        beg = row_ptr[u];
        end = row_ptr[u + 1];
    }
    while (u < n) {
        const int64_t un = u + ustep;
        int32_t nbeg = 0, nend = 0;
        if (un < n) {
            nbeg = row_ptr[un];
            nend = row_ptr[un + 1];
        }
        if (end - beg <= kLongRow) {
            const double du = d[u], pu = p[u];
            double s = 0.0;
            int32_t k = beg + sub;
            for (; k + 3 * kRowLanes < end; k += 4 * kRowLanes) {
                int32_t c[4];
                float w[4];
                double x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    c[i] = col[k + i * kRowLanes];
                    w[i] = weight[k + i * kRowLanes];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = p[c[i]];
#pragma unroll
                for (int i = 0; i < 4; ++i) s += static_cast<double>(w[i]) * x[i];
            }
            for (; k < end; k += kRowLanes) s += static_cast<double>(weight[k]) * p[col[k]];
#pragma unroll
            for (int off = kRowLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
            if (sub == 0) {
                const double y = grounded(gmask, v, u) ? 0.0 : du * pu - s;
                ap[u] = y;
                acc += pu * y;
            }
        }
        u = un;
        beg = nbeg;
        end = nend;
    }
    for (int64_t base = b; base < n; base += kBlock * nb) {
        const int64_t u = base + threadIdx.x * nb;
        const bool is_long = u < n && row_ptr[u + 1] - row_ptr[u] > kLongRow;
        const uint64_t m = __ballot(is_long);
        if ((threadIdx.x & (kWave - 1)) == 0) long_mask[threadIdx.x / kWave] = m;
        __syncthreads();
        for (int wv = 0; wv < kBlock / kWave; ++wv) {
            uint64_t bits = long_mask[wv];
            while (bits) {
                const int bit = __builtin_ctzll(bits);
                bits &= bits - 1;
                const int64_t r = base + (wv * kWave + bit) * nb;
                const int32_t beg = row_ptr[r], end = row_ptr[r + 1];
                double s = 0.0;
                for (int32_t k = beg + static_cast<int32_t>(threadIdx.x); k < end; k += kBlock)
                    s += static_cast<double>(weight[k]) * p[col[k]];
                s = block_sum(s, lds);
                if (threadIdx.x == 0) {
                    const double y = grounded(gmask, v, r) ? 0.0 : d[r] * p[r] - s;
                    ap[r] = y;
                    acc += p[r] * y;
                }
            }
        }
        __syncthreads();
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[2 * blockIdx.x] = acc;
}

__global__ void update_xr(int32_t n, int32_t v, const uint32_t* __restrict__ gmask, const Scalars* __restrict__ sc,
                          const double* __restrict__ d, double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ z, const double* __restrict__ p, const double* __restrict__ ap,
                          double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    if (sc->done) return;
    const double alpha = sc->alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (grounded(gmask, v, u)) continue;
        x[u] = x[u] + alpha * p[u];
        const double ru = r[u] - alpha * ap[u];
        const double zu = ru / d[u];
        r[u] = ru;
        z[u] = zu;
        rz += ru * zu;
        rr += ru * ru;
    }
    rz = block_sum(rz, lds);
    rr = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rz;
        part[2 * blockIdx.x + 1] = rr;
    }
}

__global__ void update_p(int32_t n, int32_t v, const uint32_t* __restrict__ gmask, const Scalars* __restrict__ sc,
                         const double* __restrict__ z, double* __restrict__ p) {
    if (sc->done) return;
    const double beta = sc->beta;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (!grounded(gmask, v, u)) p[u] = z[u] + beta * p[u];
}

// Sums the per-block partials in a fixed order and advances the CG scalars.
//   mode 0: after pcg_init (rz, rr0)    mode 1: after spmv_dot (alpha)
//   mode 2: after update_xr (beta, rr)  mode 3: after pivot_partials (rwc_v)
//   The iteration kernels return at once after the step that met the tolerance (`done`), so
//   a fixed number of launched iterations stops exactly where a host-checked loop would.
__global__ void scalars_step(const double* __restrict__ part, int nparts, Scalars* sc, int mode, double vol,
                             double tol2) {
    __shared__ double lds[kBlock / kWave];
    if ((mode == 1 || mode == 2) && sc->done) return;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    a = block_sum(a, lds);
    b = block_sum(b, lds);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        sc->rz = a;
        sc->rr0 = b;
        sc->rr = b;
        sc->beta = 0.0;
        sc->done = (b == 0.0) ? 1 : 0;
        sc->iters = 0;
    } else if (mode == 1) {
        sc->alpha = (a != 0.0) ? sc->rz / a : 0.0;
    } else if (mode == 2) {
        sc->beta = (sc->rz != 0.0) ? a / sc->rz : 0.0;
        sc->rz = a;
        sc->rr = b;
        sc->iters += 1;
        sc->done = (b <= tol2 * sc->rr0) ? 1 : 0;
    } else {
        sc->rwc_v = a / vol;
    }
}

__global__ void pivot_partials(int32_t n, const double* __restrict__ d, const double* __restrict__ h,
                               double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double s = 0.0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        s += d[u] * h[u];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

// Thread per internal index u; the caller's arrays (counts in, RWC, standard errors and
// hitting times out) are indexed by input id node_id[u].
__global__ void assemble(int32_t n, int32_t v, double vol, double l, const int32_t* __restrict__ node_id,
                         const uint64_t* __restrict__ counts, const uint64_t* __restrict__ counts_sq,
                         const double* __restrict__ d, const double* __restrict__ h, const Scalars* __restrict__ sc,
                         double* __restrict__ rwc, double* __restrict__ se, double* __restrict__ hit) {
    const double rv = sc->rwc_v;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t id = node_id[u];
        const double t = static_cast<double>(counts[id]) / l;
        if (u == v) {
            rwc[id] = rv;
        } else {
            const double a = (vol * t) / d[u];
            const double b = 2.0 * h[u];
            rwc[id] = (a - b) + rv;
        }
        if (hit) hit[id] = h[u];
        if (se) {
            double s = 0.0;
            if (u != v && l > 1.0) {
                const double c1 = static_cast<double>(counts[id]);
                const double c2 = static_cast<double>(counts_sq[id]);
                double var = (c2 - (c1 * c1) / l) / (l - 1.0);
                var = var > 0.0 ? var : 0.0;
                s = (vol / d[u]) * sqrt(var / l);
            }
            se[id] = s;
        }
    }
}

// Eq. (3) from a given estimate of diag(calL_v^{-1}) (FastChol's tau~), by input id.
__global__ void assemble_diag(int32_t n, int32_t v, double vol, const int32_t* __restrict__ node_id,
                              const double* __restrict__ diag, const double* __restrict__ d,
                              const double* __restrict__ h, const Scalars* __restrict__ sc, double* __restrict__ rwc,
                              double* __restrict__ hit) {
    const double rv = sc->rwc_v;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t id = node_id[u];
        if (u == v) {
            rwc[id] = rv;
        } else {
            const double a = (vol * diag[id]) / d[u];
            const double b = 2.0 * h[u];
            rwc[id] = (a - b) + rv;
        }
        if (hit) hit[id] = h[u];
    }
}

// Group RWC of a root set S (hitting time to the set, H_S = sum_u pi_u h_u with h solving the
// system grounded at S) and, for every node u, the estimate of H_{S + u} from the S-rooted
// forests: removing u from the grounded system is a rank-one update, so with M = L_S,
//   h' = h - (h_u / (M^-1)_uu) M^-1 e_u   and   H_{S + u} = H_S - h_u^2 / (vol (M^-1)_uu),
// and the forests' visit totals estimate d_u (M^-1)_uu by t~_u = C_u / l (as in Lemma 5.2 for
// one root), so H_{S + u} ~ H_S - d_u h_u^2 / (vol t~_u).  Nodes of S keep H_S.
__global__ void assemble_group(int32_t n, const uint32_t* __restrict__ gmask, double vol, double l,
                               const int32_t* __restrict__ node_id, const uint64_t* __restrict__ counts,
                               const double* __restrict__ d, const double* __restrict__ h,
                               const Scalars* __restrict__ sc, double* __restrict__ marginal, double* __restrict__ hit,
                               double* __restrict__ group) {
    const double hs = sc->rwc_v;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t id = node_id[u];   // caller's arrays by input id
        if (u == 0) *group = hs;
        if (hit) hit[id] = h[u];
        if (grounded(gmask, -1, u)) {
            marginal[id] = hs;
        } else {
            const double t = static_cast<double>(counts[id]) / l;
            const double q = (d[u] * (h[u] * h[u])) / (vol * t);
            marginal[id] = hs - q;
        }
    }
}

// Root set of the group estimate as a bitmap; ids out of range or repeated are reported.
__global__ void clear_words(uint32_t* __restrict__ w, int64_t count) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        w[i] = 0u;
}

__global__ void mark_roots(const int32_t* __restrict__ roots, int32_t nroots, int32_t n,
                           const int32_t* __restrict__ node_index, uint32_t* __restrict__ gmask, WsHeader* header) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nroots) return;
    const int32_t id = roots[i];
    if (id < 0 || id >= n) {
        atomicOr(&header->status, static_cast<uint32_t>(kErrNodeRange));
        return;
    }
    const int32_t r = node_index[id];
    const uint32_t bit = 1u << (r & 31);
    if (atomicOr(&gmask[r >> 5], bit) & bit) atomicOr(&header->status, static_cast<uint32_t>(kErrDupRoot));
}

__global__ void header_start(WsHeader* header) { header_begin(header); }

// After the launched iterations: the iteration count, and an error bit if the residual never
// met the tolerance.
__global__ void solve_finish(const Scalars* __restrict__ sc, WsHeader* header) {
    header->iters = sc->iters;
    if (!sc->done) atomicOr(&header->status, static_cast<uint32_t>(kErrNotConverged));
}

struct EstLayout {
    WsHeader* header;
    double *x, *r, *z, *p, *ap, *part;
    Scalars* sc;
    uint32_t* gmask;
    int64_t mask_words;
    uint32_t* cover;   // [n] components holding a root (graphs of several components)
    size_t total;
};

EstLayout carve_est(void* ws, int32_t n, bool group) {
    Carver c(ws);
    EstLayout L{};
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.x = c.take<double>(n);
    L.r = c.take<double>(n);
    L.z = c.take<double>(n);
    L.p = c.take<double>(n);
    L.ap = c.take<double>(n);
    L.part = c.take<double>(2 * kMaxBlocks);
    L.sc = c.take<Scalars>(1);
    L.mask_words = group ? (static_cast<int64_t>(n) + 31) / 32 : 0;
    L.gmask = group ? c.take<uint32_t>(L.mask_words) : nullptr;
    L.cover = group ? c.take<uint32_t>(n) : nullptr;
    L.total = c.used();
    return L;
}

// Iterations launched per call in stream-ordered mode (check_every < 0): the whole solve is
// enqueued at once, so it is bounded to keep a captured graph small.
constexpr int kMaxAsyncIter = 4096;

int check_solve_params(const rwc_solve_params* sp) {
    if (sp && sp->check_every < 0 && (sp->max_iter < 1 || sp->max_iter > kMaxAsyncIter))
        return fail(RWC_ERR_INVALID_ARG, "stream-ordered solves need max_iter in [1, %d]", kMaxAsyncIter);
    if (sp && (sp->max_iter < 0 || !(sp->tol >= 0.0)))
        return fail(RWC_ERR_INVALID_ARG, "max_iter and tol must not be negative");
    return RWC_OK;
}

// Jacobi-PCG on the system grounded at v (or at the set in L.gmask): x solves L_G x = d_{-G}.
// Host-checked mode reads the scalars every `check` iterations; stream-ordered mode
// (check < 0) launches max_iter iterations, which stop on the device at convergence, and
// leaves the outcome in the workspace header.
int pivot_solve(const rwc_csr* g, int32_t v, const EstLayout& L, const rwc_solve_params* sp, int32_t* iters,
                hipStream_t s, bool* async_out) {
    const int32_t n = g->n;
    const double tol = (sp && sp->tol > 0) ? sp->tol : 1e-12;
    const bool async = sp && sp->check_every < 0;
    const int max_iter = (sp && sp->max_iter > 0) ? sp->max_iter : (async ? 0 : 20000);
    const int check = (sp && sp->check_every > 0) ? sp->check_every : 16;
    const double tol2 = tol * tol;
    const unsigned nb = blocks_for(n, kBlock) < kMaxBlocks ? blocks_for(n, kBlock) : kMaxBlocks;
    const int64_t spmv_threads = static_cast<int64_t>(n) * kRowLanes;
    const unsigned nb_spmv = blocks_for(spmv_threads, kBlock) < kMaxBlocks ? blocks_for(spmv_threads, kBlock) : kMaxBlocks;
    *async_out = async;

    hipLaunchKernelGGL(pcg_init, dim3(nb), dim3(kBlock), 0, s, n, v, L.gmask, g->strength, L.x, L.r, L.z, L.p, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 0, g->vol, tol2);
    auto iteration = [&]() {
        hipLaunchKernelGGL(spmv_dot, dim3(nb_spmv), dim3(kBlock), 0, s, n, v, L.gmask, L.sc, g->row_ptr, g->col,
                           g->weight, g->strength, L.p, L.ap, L.part);
        hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb_spmv), L.sc, 1,
                           g->vol, tol2);
        hipLaunchKernelGGL(update_xr, dim3(nb), dim3(kBlock), 0, s, n, v, L.gmask, L.sc, g->strength, L.x, L.r, L.z,
                           L.p, L.ap, L.part);
        hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 2, g->vol,
                           tol2);
        hipLaunchKernelGGL(update_p, dim3(nb), dim3(kBlock), 0, s, n, v, L.gmask, L.sc, L.z, L.p);
    };
    if (async) {
        for (int it = 0; it < max_iter; ++it) iteration();
        hipLaunchKernelGGL(solve_finish, dim3(1), dim3(1), 0, s, L.sc, L.header);
        RWC_HIP(hipGetLastError());
        if (iters) *iters = -1;
        return RWC_OK;
    }
    RWC_HIP(hipGetLastError());
    Scalars host{};
    RWC_HIP(hipMemcpyAsync(&host, L.sc, sizeof(host), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    int launched = 0;
    while (!host.done && launched < max_iter) {
        const int chunk = (max_iter - launched) < check ? (max_iter - launched) : check;
        for (int c = 0; c < chunk; ++c) iteration();
        RWC_HIP(hipGetLastError());
        launched += chunk;
        RWC_HIP(hipMemcpyAsync(&host, L.sc, sizeof(host), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(solve_finish, dim3(1), dim3(1), 0, s, L.sc, L.header);
    if (iters) *iters = host.iters;
    if (!host.done)
        return fail(RWC_ERR_NOT_CONVERGED, "pivot solve: relative residual %.3e after %d iterations",
                    host.rr > 0 ? std::sqrt(host.rr / host.rr0) : 0.0, host.iters);
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_estimate_workspace(const rwc_csr* g, size_t* bytes) {
    clear_error();
    if (!g || !bytes) return fail(RWC_ERR_INVALID_ARG, "g and bytes must not be null");
    *bytes = carve_est(nullptr, g->n, false).total;
    return RWC_OK;
}

extern "C" int rwc_estimate(const rwc_csr* g, const uint64_t* counts, const uint64_t* counts_sq, int64_t l,
                            const rwc_solve_params* sp, double* rwc, double* hit, double* stderr_out, int32_t* iters,
                            void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g || !counts || !rwc) return fail(RWC_ERR_INVALID_ARG, "g, counts and rwc must not be null");
    RWC_CHECK(require_connected(g, "rwc_estimate (the pivot solve)"));
    if (l < 1) return fail(RWC_ERR_INVALID_ARG, "l must be positive");
    if (stderr_out && !counts_sq) return fail(RWC_ERR_INVALID_ARG, "stderr needs counts_sq");
    RWC_CHECK(check_solve_params(sp));
    const int32_t n = g->n;
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_est(nullptr, n, false).total));
    EstLayout L = carve_est(ws, n, false);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int v = g->pivot_index;
    const unsigned nb = blocks_for(n, kBlock) < kMaxBlocks ? blocks_for(n, kBlock) : kMaxBlocks;
    hipLaunchKernelGGL(header_start, dim3(1), dim3(1), 0, s, L.header);
    bool async = false;
    RWC_CHECK(pivot_solve(g, v, L, sp, iters, s, &async));
    hipLaunchKernelGGL(pivot_partials, dim3(nb), dim3(kBlock), 0, s, n, g->strength, L.x, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 3, g->vol, 0.0);
    hipLaunchKernelGGL(assemble, dim3(nb), dim3(kBlock), 0, s, n, v, g->vol, static_cast<double>(l), g->node_id, counts,
                       counts_sq, g->strength, L.x, L.sc, rwc, stderr_out, hit);
    RWC_HIP(hipGetLastError());
    if (!async) RWC_HIP(hipStreamSynchronize(s));
    return RWC_OK;
}

extern "C" int rwc_estimate_diag(const rwc_csr* g, const double* diag, const rwc_solve_params* sp, double* rwc,
                                 double* hit, int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g || !diag || !rwc) return fail(RWC_ERR_INVALID_ARG, "g, diag and rwc must not be null");
    RWC_CHECK(require_connected(g, "rwc_estimate_diag (the pivot solve)"));
    RWC_CHECK(check_solve_params(sp));
    const int32_t n = g->n;
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_est(nullptr, n, false).total));
    EstLayout L = carve_est(ws, n, false);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int v = g->pivot_index;
    const unsigned nb = blocks_for(n, kBlock) < kMaxBlocks ? blocks_for(n, kBlock) : kMaxBlocks;
    hipLaunchKernelGGL(header_start, dim3(1), dim3(1), 0, s, L.header);
    bool async = false;
    RWC_CHECK(pivot_solve(g, v, L, sp, iters, s, &async));
    hipLaunchKernelGGL(pivot_partials, dim3(nb), dim3(kBlock), 0, s, n, g->strength, L.x, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 3, g->vol, 0.0);
    hipLaunchKernelGGL(assemble_diag, dim3(nb), dim3(kBlock), 0, s, n, v, g->vol, g->node_id, diag, g->strength, L.x,
                       L.sc, rwc, hit);
    RWC_HIP(hipGetLastError());
    if (!async) RWC_HIP(hipStreamSynchronize(s));
    return RWC_OK;
}

extern "C" int rwc_estimate_group_workspace(const rwc_csr* g, size_t* bytes) {
    clear_error();
    if (!g || !bytes) return fail(RWC_ERR_INVALID_ARG, "g and bytes must not be null");
    *bytes = carve_est(nullptr, g->n, true).total;
    return RWC_OK;
}

extern "C" int rwc_estimate_group(const rwc_csr* g, const int32_t* roots, int32_t num_roots, const uint64_t* counts,
                                  int64_t l, const rwc_solve_params* sp, double* group_rwc, double* marginal,
                                  double* hit, int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g || !roots || !counts || !group_rwc || !marginal)
        return fail(RWC_ERR_INVALID_ARG, "g, roots, counts, group_rwc and marginal must not be null");
    if (l < 1) return fail(RWC_ERR_INVALID_ARG, "l must be positive");
    const int32_t n = g->n;
    if (num_roots < 1 || num_roots >= n) return fail(RWC_ERR_INVALID_ARG, "num_roots must be in [1, n - 1]");
    RWC_CHECK(check_solve_params(sp));
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_est(nullptr, n, true).total));
    EstLayout L = carve_est(ws, n, true);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned nb = blocks_for(n, kBlock) < kMaxBlocks ? blocks_for(n, kBlock) : kMaxBlocks;
    hipLaunchKernelGGL(header_start, dim3(1), dim3(1), 0, s, L.header);
    hipLaunchKernelGGL(clear_words, dim3(blocks_for(L.mask_words, kBlock)), dim3(kBlock), 0, s, L.gmask, L.mask_words);
    hipLaunchKernelGGL(mark_roots, dim3(blocks_for(num_roots, kBlock)), dim3(kBlock), 0, s, roots, num_roots, n,
                       g->node_index, L.gmask, L.header);
    if (g->components > 1) check_root_cover(*g, roots, num_roots, L.cover, L.gmask, L.header, s);
    if (!(sp && sp->check_every < 0)) {
        // host-checked mode: a bad root set would leave the system singular, so stop here
        WsHeader h{};
        RWC_HIP(hipMemcpyAsync(&h, L.header, sizeof(h), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
        RWC_CHECK(device_error_to_status(h.status));
    }
    bool async = false;
    RWC_CHECK(pivot_solve(g, -1, L, sp, iters, s, &async));
    hipLaunchKernelGGL(pivot_partials, dim3(nb), dim3(kBlock), 0, s, n, g->strength, L.x, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 3, g->vol, 0.0);
    hipLaunchKernelGGL(assemble_group, dim3(nb), dim3(kBlock), 0, s, n, L.gmask, g->vol, static_cast<double>(l),
                       g->node_id, counts, g->strength, L.x, L.sc, marginal, hit, group_rwc);
    RWC_HIP(hipGetLastError());
    if (!async) {
        // the root set is validated on the device: report it with the synchronous result
        WsHeader h{};
        RWC_HIP(hipMemcpyAsync(&h, L.header, sizeof(h), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
        return device_error_to_status(h.status);
    }
    return RWC_OK;
}

// ---------------------------------------------------------------------------------------
// rwc_estimate_static: rwc_estimate over a fixed device array instead of a caller workspace,
// for callers that cannot allocate.  `scratch` is a host-side stand-in for the array in host
// code; its device address (one per GPU) comes from hipGetSymbolAddress on the first call on
// each device and is the only handle passed to kernels.
// ---------------------------------------------------------------------------------------
namespace rwc {
namespace {
constexpr size_t kStaticScratchBytes = size_t{128} << 20;   // 128 MiB: graphs up to ~3.35 M nodes
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

int static_scratch(void** out) {
    static std::mutex mu;
    static void* ptrs[64] = {};
    int dev = 0;
    RWC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(RWC_ERR_HIP, "device %d out of the supported range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        RWC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(RWC_ERR_HIP, "hipGetSymbolAddress returned a null address");
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return RWC_OK;
}
}  // namespace
}  // namespace rwc

extern "C" int rwc_estimate_static(const rwc_csr* g, const uint64_t* counts, const uint64_t* counts_sq, int64_t l,
                                   const rwc_solve_params* sp, double* rwc_out, double* hit, double* stderr_out,
                                   int32_t* iters, void* stream) {
    clear_error();
    if (!g) return fail(RWC_ERR_INVALID_ARG, "g must not be null");
    RWC_CHECK(require_connected(g, "rwc_estimate_static (the pivot solve)"));
    if (sp && sp->check_every < 0)
        return fail(RWC_ERR_INVALID_ARG, "rwc_estimate_static runs the host-checked solve only");
    const size_t need = carve_est(nullptr, g->n, false).total;
    if (need > kStaticScratchBytes)
        return fail(RWC_ERR_TOO_LARGE, "rwc_estimate_static: n = %d needs %zu bytes of scratch, the fixed array has %zu",
                    g->n, need, kStaticScratchBytes);
    void* ws = nullptr;
    RWC_CHECK(static_scratch(&ws));
    return rwc_estimate(g, counts, counts_sq, l, sp, rwc_out, hit, stderr_out, iters, ws, kStaticScratchBytes, stream);
}
