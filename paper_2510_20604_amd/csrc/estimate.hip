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

#include "common.hpp"
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
    double rwc_v;   // RWC of the pivot
};

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

__global__ void pcg_init(int32_t n, int32_t v, const double* __restrict__ d, double* __restrict__ x,
                         double* __restrict__ r, double* __restrict__ z, double* __restrict__ p,
                         double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double rz = 0.0, rr = 0.0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double ru = (u == v) ? 0.0 : d[u];
        const double zu = (u == v) ? 0.0 : ru / d[u];
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
// power-law graphs, land in different blocks.  Eight lanes share a short row (strided over its
// entries, then a shuffle reduction); rows longer than kLongRow are left out of that pass and
// then taken one at a time, in order, by the whole block.
constexpr int kRowLanes = 8;
constexpr int kLongRow = 16 * kRowLanes;

__global__ void spmv_dot(int32_t n, int32_t v, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const float* __restrict__ weight, const double* __restrict__ d, const double* __restrict__ p,
                         double* __restrict__ ap, double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    __shared__ uint64_t long_mask[kBlock / kWave];
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
                const double y = (u == v) ? 0.0 : du * pu - s;
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
                    const double y = (r == v) ? 0.0 : d[r] * p[r] - s;
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

__global__ void update_xr(int32_t n, int32_t v, const Scalars* __restrict__ sc, const double* __restrict__ d,
                          double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                          const double* __restrict__ p, const double* __restrict__ ap, double* __restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    const double alpha = sc->alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (u == v) continue;
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

__global__ void update_p(int32_t n, int32_t v, const Scalars* __restrict__ sc, const double* __restrict__ z,
                         double* __restrict__ p) {
    const double beta = sc->beta;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (u != v) p[u] = z[u] + beta * p[u];
}

// Sums the per-block partials in a fixed order and advances the CG scalars.
//   mode 0: after pcg_init (rz, rr0)    mode 1: after spmv_dot (alpha)
//   mode 2: after update_xr (beta, rr)  mode 3: after pivot_partials (rwc_v)
__global__ void scalars_step(const double* __restrict__ part, int nparts, Scalars* sc, int mode, double vol) {
    __shared__ double lds[kBlock / kWave];
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
    } else if (mode == 1) {
        sc->alpha = (a != 0.0) ? sc->rz / a : 0.0;
    } else if (mode == 2) {
        sc->beta = (sc->rz != 0.0) ? a / sc->rz : 0.0;
        sc->rz = a;
        sc->rr = b;
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

__global__ void assemble(int32_t n, int32_t v, double vol, double l, const uint64_t* __restrict__ counts,
                         const uint64_t* __restrict__ counts_sq, const double* __restrict__ d,
                         const double* __restrict__ h, const Scalars* __restrict__ sc, double* __restrict__ rwc,
                         double* __restrict__ se) {
    const double rv = sc->rwc_v;
    for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double t = static_cast<double>(counts[u]) / l;
        if (u == v) {
            rwc[u] = rv;
        } else {
            const double a = (vol * t) / d[u];
            const double b = 2.0 * h[u];
            rwc[u] = (a - b) + rv;
        }
        if (se) {
            double s = 0.0;
            if (u != v && l > 1.0) {
                const double c1 = static_cast<double>(counts[u]);
                const double c2 = static_cast<double>(counts_sq[u]);
                double var = (c2 - (c1 * c1) / l) / (l - 1.0);
                var = var > 0.0 ? var : 0.0;
                s = (vol / d[u]) * sqrt(var / l);
            }
            se[u] = s;
        }
    }
}

struct EstLayout {
    double *x, *r, *z, *p, *ap, *part;
    Scalars* sc;
    size_t total;
};

EstLayout carve_est(void* ws, int32_t n) {
    Carver c(ws);
    EstLayout L{};
    L.x = c.take<double>(n);
    L.r = c.take<double>(n);
    L.z = c.take<double>(n);
    L.p = c.take<double>(n);
    L.ap = c.take<double>(n);
    L.part = c.take<double>(2 * kMaxBlocks);
    L.sc = c.take<Scalars>(1);
    L.total = c.used();
    return L;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_estimate_workspace(const rwc_csr* g, size_t* bytes) {
    clear_error();
    if (!g || !bytes) return fail(RWC_ERR_INVALID_ARG, "g and bytes must not be null");
    *bytes = carve_est(nullptr, g->n).total;
    return RWC_OK;
}

extern "C" int rwc_estimate(const rwc_csr* g, const uint64_t* counts, const uint64_t* counts_sq, int64_t l,
                            const rwc_solve_params* sp, double* rwc, double* hit, double* stderr_out, int32_t* iters,
                            void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g || !counts || !rwc) return fail(RWC_ERR_INVALID_ARG, "g, counts and rwc must not be null");
    if (l < 1) return fail(RWC_ERR_INVALID_ARG, "l must be positive");
    if (stderr_out && !counts_sq) return fail(RWC_ERR_INVALID_ARG, "stderr needs counts_sq");
    const int32_t n = g->n;
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_est(nullptr, n).total));
    EstLayout L = carve_est(ws, n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double tol = (sp && sp->tol > 0) ? sp->tol : 1e-12;
    const int max_iter = (sp && sp->max_iter > 0) ? sp->max_iter : 20000;
    const int check = (sp && sp->check_every > 0) ? sp->check_every : 16;
    const int v = g->pivot;
    const unsigned nb = blocks_for(n, kBlock) < kMaxBlocks ? blocks_for(n, kBlock) : kMaxBlocks;
    const int64_t spmv_threads = static_cast<int64_t>(n) * kRowLanes;
    const unsigned nb_spmv = blocks_for(spmv_threads, kBlock) < kMaxBlocks ? blocks_for(spmv_threads, kBlock) : kMaxBlocks;

    hipLaunchKernelGGL(pcg_init, dim3(nb), dim3(kBlock), 0, s, n, v, g->strength, L.x, L.r, L.z, L.p, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 0, g->vol);
    RWC_HIP(hipGetLastError());
    Scalars host{};
    RWC_HIP(hipMemcpyAsync(&host, L.sc, sizeof(host), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    const double bnorm2 = host.rr0;
    int it = 0;
    bool converged = (bnorm2 == 0.0);
    while (!converged && it < max_iter) {
        const int chunk = (max_iter - it) < check ? (max_iter - it) : check;
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(spmv_dot, dim3(nb_spmv), dim3(kBlock), 0, s, n, v, g->row_ptr, g->col, g->weight,
                               g->strength, L.p, L.ap, L.part);
            hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb_spmv), L.sc, 1,
                               g->vol);
            hipLaunchKernelGGL(update_xr, dim3(nb), dim3(kBlock), 0, s, n, v, L.sc, g->strength, L.x, L.r, L.z, L.p,
                               L.ap, L.part);
            hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 2, g->vol);
            hipLaunchKernelGGL(update_p, dim3(nb), dim3(kBlock), 0, s, n, v, L.sc, L.z, L.p);
        }
        RWC_HIP(hipGetLastError());
        it += chunk;
        RWC_HIP(hipMemcpyAsync(&host, L.sc, sizeof(host), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
        converged = host.rr <= tol * tol * bnorm2;
    }
    if (iters) *iters = it;
    if (!converged)
        return fail(RWC_ERR_NOT_CONVERGED, "pivot solve: relative residual %.3e after %d iterations",
                    host.rr > 0 ? std::sqrt(host.rr / bnorm2) : 0.0, it);
    hipLaunchKernelGGL(pivot_partials, dim3(nb), dim3(kBlock), 0, s, n, g->strength, L.x, L.part);
    hipLaunchKernelGGL(scalars_step, dim3(1), dim3(kBlock), 0, s, L.part, static_cast<int>(nb), L.sc, 3, g->vol);
    hipLaunchKernelGGL(assemble, dim3(nb), dim3(kBlock), 0, s, n, v, g->vol, static_cast<double>(l), counts, counts_sq,
                       g->strength, L.x, L.sc, rwc, stderr_out);
    if (hit) RWC_HIP(hipMemcpyAsync(hit, L.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipStreamSynchronize(s));
    return RWC_OK;
}
