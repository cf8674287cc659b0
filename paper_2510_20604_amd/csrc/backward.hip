// rwc_backward: gradient of l(w) = sum_j g_j RWC_j with respect to the edge weights.
//
// RWC_j = vol L^+_jj - 2 (L^+ d)_j + d^T L^+ d / vol (Eq. (2) with the pseudo-inverse
// identity of Section 3).  With dL/dw_e = b_e b_e^T (b_e from the incidence matrix of
// Section 2.2), dL^+/dw_e = -L^+ b_e b_e^T L^+, dd/dw_e = e_a + e_b and dvol/dw_e = 2:
//   dl/dw_e = 2 trGL - vol Q_e + 2 D_A D_B - 2 S_A + G ((2 S_B - D_B^2)/vol - 2 dLd/vol^2)
// with A = L^+ g, B = L^+ d, G = sum g, trGL = sum_j g_j L^+_jj, dLd = d^T B,
// Q_e = sum_j g_j (L^+ b_e)_j^2, D_X = X_a - X_b, S_X = X_a + X_b for e = (a, b).
//
// Q_e and trGL are carried by probe columns y_i with coefficients c_i:
//   Q_e ~ sum_i c_i (b_e^T L^+ y_i)^2,   trGL ~ sum_i c_i y_i^T L^+ y_i.
// Exact mode: one column per target j, y = sqrt|g_j| e_j, c = sign(g_j).  Sketch mode (a
// Johnson-Lindenstrauss / Hutchinson estimate): k Rademacher columns per sign class of g,
// y_i = sqrt(|g|) r_i on the targets of that class, c_i = +-1/k.  The same columns give Q^ and
// trGL^, which keeps sum_e w_e dl/dw_e = 0 exactly.
//
// All columns [g, d, y_1..y_P] are centred and solved together on the grounded Laplacian L_v
// (row and column of the pivot removed) by a batched Jacobi-preconditioned conjugate gradient:
// FP64 iterate and residual, FP32 search directions (the SpMM gathers half the bytes), FP64
// accumulation of every product and dot.  Because the stored FP32 direction is exactly what
// the operator is applied to, x and r stay consistent; the step and direction updates use the
// residual-based (flexible) formulas alpha = r.p / p.Ap and beta = z'.(r' - r) / z.r, which
// tolerate the rounded directions.  Solutions are centred at the end (L^+ y = z - mean(z)).
// This file is compiled without FMA contraction.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace rwc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxWaves = 8192;   // bound of the per-wave partial arrays
constexpr int kUpdateSlots = 2048;   // partial slots per column of bpcg_update (<= kMaxWaves)
constexpr int kDirSlots = 8192;      // partial slots per column of bpcg_init and bpcg_direction (<= kMaxWaves)

__global__ void header_start(WsHeader* header) { header_begin(header); }

__global__ void fill_zero(double* __restrict__ x, int64_t count) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        x[i] = 0.0;
}

struct ColScalars {
    double alpha, beta, zr, rr, rr0, zr_new, zro, rp, pap;
    int32_t done;
    int32_t pad;
};

// Batched-PCG progress: columns converged so far, and iterations run.  Once every column is
// done, the iteration's kernels return at once (the host looks only every few iterations).
struct BpcgState {
    int32_t ndone;
    int32_t iters;
};

// ----------------------------------------------------------------- RHS ---------------
// The right-hand sides are built on the device from the dense g: column 0 is g, column 1 is d,
// columns 2.. are the probe columns y_i, then every column is centred.
//   Exact mode (k = 0): the nonzeros of g in ascending node order get columns 2, 3, ...;
//   y = sqrt|g_u| e_u with coefficient sign(g_u).
//   Sketch mode: k columns per sign class of g present (positive class first); probe i of
//   class s (0 positive, 1 negative) is numbered s k + i, y_u = +-sqrt|g_u| on the nodes of
//   its class with the sign from bit 0 of Philox word 0 on (s k + i, u, 0, 2^32 - 1) under
//   the probe key, coefficient +-1/k.
struct ProbeSpec {
    int32_t k;          // 0: exact
    int32_t pos;        // 1 if the positive class is present (it then takes the first k columns)
    uint32_t s0, s1;    // probe key
};

// Class of g_u's sign, and the first probe column of that class.
__device__ __forceinline__ int32_t class_first_column(const ProbeSpec& ps, double gu) {
    return 2 + ((gu > 0.0 || !ps.pos) ? 0 : ps.k);
}

__device__ __forceinline__ double probe_entry(const ProbeSpec& ps, double gu, uint32_t u, int32_t i) {
    const uint32_t cls = gu > 0.0 ? 0u : 1u;
    const uint64_t x = philox_x64(cls * static_cast<uint32_t>(ps.k) + static_cast<uint32_t>(i), u, 0u, 0xFFFFFFFFu,
                                  ps.s0, ps.s1);
    const double a = sqrt(fabs(gu));
    return (x & 1ull) ? -a : a;
}

// Per block over its contiguous row range: number of positive, negative, nonzero and
// non-finite entries of g and their sum (thread sums, then a fixed tree).
struct GPart {
    double sum;
    int32_t npos, nneg, nnz, nbad;
};

__device__ double block_sum(double v, double* lds);

__global__ void g_partials(int32_t n, int32_t rows_per_block, const double* __restrict__ g, GPart* __restrict__ out) {
    __shared__ double lds[kBlock];
    __shared__ int32_t cnt[4];
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * rows_per_block;
    const int64_t hi = lo + rows_per_block < n ? lo + rows_per_block : n;
    double sum = 0.0;
    int32_t np = 0, nn = 0, nb = 0;
    for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
        const double gu = g[u];
        if (!isfinite(gu)) {
            ++nb;
            continue;
        }
        np += gu > 0.0;
        nn += gu < 0.0;
        sum += gu;
    }
    sum = block_sum(sum, lds);
    atomicAdd(&cnt[0], np);
    atomicAdd(&cnt[1], nn);
    atomicAdd(&cnt[2], nb);
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = GPart{sum, cnt[0], cnt[1], cnt[0] + cnt[1], cnt[2]};
}

// Exact mode: the rank of every nonzero of g among all nonzeros in node order (block b starts
// at base[b]; within the block a scan over chunks of kBlock rows), and its coefficient.
__global__ void rank_nonzeros(int32_t n, int32_t rows_per_block, const double* __restrict__ g,
                              const int32_t* __restrict__ base, int32_t* __restrict__ rank, double* __restrict__ coef) {
    __shared__ int32_t scan[kBlock];
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * rows_per_block;
    const int64_t hi = lo + rows_per_block < n ? lo + rows_per_block : n;
    int32_t carry = base[blockIdx.x];
    for (int64_t u0 = lo; u0 < hi; u0 += kBlock) {
        const int64_t u = u0 + threadIdx.x;
        const double gu = u < hi ? g[u] : 0.0;
        const int32_t f = gu != 0.0 ? 1 : 0;
        scan[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {   // inclusive Hillis-Steele scan
            const int32_t add = static_cast<int>(threadIdx.x) >= off ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += add;
            __syncthreads();
        }
        if (u < hi) {
            const int32_t r = f ? carry + scan[threadIdx.x] - 1 : -1;
            rank[u] = r;
            if (f) coef[2 + r] = gu > 0.0 ? 1.0 : -1.0;
        }
        carry += scan[kBlock - 1];
        __syncthreads();
    }
}

// Row u of Y is internal index u; g, rank and the probe keys use its input id node_id[u].
__global__ void rhs_fill(int32_t n, int32_t R, ProbeSpec ps, const double* __restrict__ g,
                         const int32_t* __restrict__ node_id, const double* __restrict__ d,
                         const int32_t* __restrict__ rank, double* __restrict__ Y) {
    const int64_t total = static_cast<int64_t>(n) * R;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t u = i / R;
        const int32_t c = static_cast<int32_t>(i - u * R);
        const int32_t id = node_id[u];
        const double gu = g[id];
        double v = 0.0;
        if (c == 0) {
            v = gu;
        } else if (c == 1) {
            v = d[u];
        } else if (gu != 0.0) {
            if (ps.k == 0) {
                if (rank[id] == c - 2) v = sqrt(fabs(gu));
            } else {
                const int32_t first = class_first_column(ps, gu);
                if (c >= first && c < first + ps.k) v = probe_entry(ps, gu, static_cast<uint32_t>(id), c - first);
            }
        }
        Y[i] = v;
    }
}

// ------------------------------------------------------------ batched PCG ------------
// The FP32 search directions P are stored in blocks of 64 columns: block b holds columns
// 64b .. 64b + w_b - 1 (w_b = min(64, R - 64b)) of every row, row-major with row stride w_b,
// and starts at float 64 b n.  A row of a full block is 256 aligned bytes, two L2 lines, so the
// SpMM's random gather of a neighbour's row touches two lines of HBM instead of three for an
// R-wide row; the narrow last block (2 columns for 64 probes: 8 B per row) is small enough to
// stay in the Infinity Cache.
__device__ __forceinline__ int64_t p_block_base(int32_t b, int64_t n) { return static_cast<int64_t>(b) * kWave * n; }
__device__ __forceinline__ int32_t p_block_width(int32_t b, int32_t R) {
    return (R - b * kWave) < kWave ? (R - b * kWave) : kWave;
}
__device__ __forceinline__ int64_t p_index(int64_t u, int32_t c, int32_t R, int64_t n) {
    const int32_t b = c / kWave;
    return p_block_base(b, n) + u * p_block_width(b, R) + (c - b * kWave);
}

// Per-wave partial dot products of the PCG kernels: value k of column c from wave (or partial
// slot) w of nw lives at (k R + c) nw + w, so the reduction of one column reads contiguous
// memory.
__device__ __forceinline__ int64_t part_index(int k, int32_t c, int64_t w, int32_t R, int64_t nw) {
    return (static_cast<int64_t>(k) * R + c) * nw + w;
}

// partials each thread of bpcg_scalars loads at once
constexpr int kScalarBatch = 8;

// The residual starts as the right-hand side (zero on row v), X = 0 and P = z = r / d; the
// partial dots z.r and r.r, and r.P with P as stored.  One thread per (row, column) element
// as in bpcg_update (the thread count is a multiple of R; thread t keeps column t mod R and
// fills partial slot t / R).
__global__ void bpcg_init(int32_t n, int32_t v, int32_t R, const double* __restrict__ d, double* __restrict__ Y,
                          double* __restrict__ X, float* __restrict__ P32, double* __restrict__ part,
                          double* __restrict__ rp_part, BpcgState* __restrict__ st) {
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (t == 0) *st = BpcgState{0, 0};
    const int64_t rows_step = static_cast<int64_t>(gridDim.x) * blockDim.x / R;
    const int32_t c = static_cast<int32_t>(t % R);
    double zr = 0.0, rr = 0.0, rp = 0.0;
    for (int64_t u = t / R; u < n; u += rows_step) {
        const int64_t i = u * R + c;
        const double r = (u == v) ? 0.0 : Y[i];
        const double z = (u == v) ? 0.0 : r / d[u];
        Y[i] = r;   // Y becomes the residual
        X[i] = 0.0;
        const float p = static_cast<float>(z);
        P32[p_index(u, c, R, n)] = p;
        zr += z * r;
        rr += r * r;
        rp += r * static_cast<double>(p);
    }
    const int64_t slot = t / R;
    part[part_index(0, c, slot, R, rows_step)] = zr;
    part[part_index(1, c, slot, R, rows_step)] = rr;
    rp_part[part_index(0, c, slot, R, rows_step)] = rp;
}

// AP = L_v P (FP32 P promoted, FP64 sums) and the partial dot P.AP per column (r.P comes from
// the kernel that writes P).
//
// The gathers of neighbour rows of P reach HBM bandwidth only with many of them in flight, so a
// wave keeps kChunk of them in flight at every step, whatever rows their entries belong to.  The CSR entries are
// cut into one contiguous segment per wave, balanced on the cost nnz + kRowCost n (a wave
// runs one round per kChunk entries or per kQueue row ends, whichever comes first).  A wave
// walks its segment in rounds: the round's entries, up to kChunk of them, have their rows of P
// gathered together and added in entry order to the running sum of the row they belong to.
// A row that ends in a round leaves its sum in a small per-wave LDS queue, and is finished
// (AP row, P.AP) in the next round while that round's gathers are in flight.  A row cut by a
// segment boundary leaves the sum of its entries in each segment in a slot: the head slot of
// a segment that starts inside the row, the tail slot of the segment the row starts in;
// spmm_fixup adds them in segment order and finishes the row.  Lane l holds the columns
// c0 + l + 64 j (j < kColPass), so one pass over the entries serves up to 128 columns.  Every
// row has an entry (the adjoint needs a connected graph of two or more nodes), and row v of P
// is zero, so its column entries need no test.
constexpr int kColPass = 2;
constexpr int kChunk = 16;     // gathers in flight per wave
constexpr int kQueue = 8;      // finished rows a wave holds before writing them out
constexpr int kRowCost = 10;   // the cost of a row, in entries, for the segment balance
constexpr int kSegMinCost = 64;   // the least cost of a segment (small graphs use fewer waves)

// Segments the CSR is cut into: at most `waves`, each of cost at least kSegMinCost.
int32_t spmm_segments(int64_t nnz, int32_t n, int64_t waves) {
    const int64_t by_cost = (nnz + static_cast<int64_t>(kRowCost) * n) / kSegMinCost;
    const int64_t s = by_cost < waves ? by_cost : waves;
    return static_cast<int32_t>(s < 1 ? 1 : s);
}

// Segment s of W starts at entry seg_k[s], in row seg_row[s] (s = W: nnz and n).  The cost of
// the rows before r and of the entries before k in row r is row_ptr[r] + kRowCost (r + 1) +
// (k - row_ptr[r]) (a row's cost comes before its entries); segment s starts where it reaches
// s (nnz + kRowCost n) / W.
__global__ void spmm_bounds(int32_t n, int32_t nnz, int32_t W, const int32_t* __restrict__ row_ptr,
                            int32_t* __restrict__ seg_k, int32_t* __restrict__ seg_row) {
    const int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (s > W) return;
    const int64_t total = static_cast<int64_t>(nnz) + static_cast<int64_t>(kRowCost) * n;
    const int64_t T = total * s / W;
    int32_t lo = 0, hi = n;   // largest r with row_ptr[r] + kRowCost r <= T
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] + static_cast<int64_t>(kRowCost) * mid <= T)
            lo = mid;
        else
            hi = mid - 1;
    }
    int32_t k = nnz, r = n;
    if (lo < n) {
        const int64_t into = T - row_ptr[lo] - static_cast<int64_t>(kRowCost) * (lo + 1);
        k = row_ptr[lo] + static_cast<int32_t>(into > 0 ? into : 0);
        if (k > row_ptr[lo + 1]) k = row_ptr[lo + 1];
        r = lo;
        while (r < n && row_ptr[r + 1] <= k) ++r;   // the row that holds entry k
    }
    seg_k[s] = k;
    seg_row[s] = r;
}

// End of row x (row_ptr[x + 1]), or past every entry for x >= n.
__device__ __forceinline__ int32_t row_end(const int32_t* __restrict__ row_ptr, int32_t n, int64_t x) {
    return x < n ? row_ptr[x + 1] : INT32_MAX;
}

__device__ __forceinline__ int32_t lane_int(int32_t x, int32_t l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float lane_float(float x, int32_t l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_double(double x, int32_t l) {
    const int64_t b = __double_as_longlong(x);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int32_t>(b), l));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int32_t>(b >> 32), l));
    return __longlong_as_double(static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo));
}

// Finishes row u from its neighbour sums s (this lane's columns c0 + lane + 64 j): AP row and
// the dot P.AP.
struct RowFinish {
    int32_t n, v, R, c0, lane;
    const double* __restrict__ d;
    const float* __restrict__ P32;
    double* __restrict__ AP;
};

// Writes out the rows q0 .. q0 + qn - 1 (qn <= kQueue) whose sums the queue holds, in order;
// their own inputs are all loaded before the first is finished.
__device__ __forceinline__ void finish_queued(const RowFinish& f, int32_t q0, int32_t qn,
                                              const double (*queue)[kColPass * kWave], double* pap) {
    // lane i < qn holds d of row q0 + i
    const double dv = f.d[q0 + (f.lane < qn ? f.lane : qn - 1)];
    float pu[kQueue][kColPass];
#pragma unroll
    for (int i = 0; i < kQueue; ++i) {
        if (i >= qn) continue;
        const int64_t u = q0 + i;
#pragma unroll
        for (int j = 0; j < kColPass; ++j) {
            // lanes past column R - 1 load column R - 1 (unused), so no load is predicated
            const int32_t c = f.c0 + f.lane + j * kWave < f.R ? f.c0 + f.lane + j * kWave : f.R - 1;
            pu[i][j] = f.P32[p_index(u, c, f.R, f.n)];
        }
    }
#pragma unroll
    for (int i = 0; i < kQueue; ++i) {
        if (i >= qn) continue;
        const int64_t u = q0 + i;
#pragma unroll
        for (int j = 0; j < kColPass; ++j) {
            const int32_t c = f.c0 + f.lane + j * kWave;
            if (c >= f.R) continue;
            const double p = static_cast<double>(pu[i][j]);
            const double y = (u == f.v) ? 0.0 : lane_double(dv, i) * p - queue[i][f.lane + j * kWave];
            f.AP[u * f.R + c] = y;
            pap[j] += p * y;
        }
    }
}

__global__ void bpcg_spmm(int32_t n, int32_t v, int32_t R, int32_t nnz, int32_t W,
                          const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                          const float* __restrict__ weight, const double* __restrict__ d,
                          const float* __restrict__ P32, const int32_t* __restrict__ seg_k,
                          const int32_t* __restrict__ seg_row, double* __restrict__ AP, double* __restrict__ cut,
                          double* __restrict__ part, const BpcgState* __restrict__ st) {
    __shared__ double queue_all[kWavesPerBlock][kQueue][kColPass * kWave];
    if (st->ndone == R) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // uniform: the segment walk is scalar
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wib;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    double (*queue)[kColPass * kWave] = queue_all[wib];
    for (int32_t c0 = 0; c0 < R; c0 += kColPass * kWave) {
        double pap[kColPass];
#pragma unroll
        for (int j = 0; j < kColPass; ++j) pap[j] = 0.0;
        const RowFinish f{n, v, R, c0, lane, d, P32, AP};
        if (wave < W) {
            const int32_t k0 = seg_k[wave], k1 = seg_k[wave + 1];
            int32_t r = seg_row[wave];                     // the row holding entry k0
            int32_t rstart = r < n ? row_ptr[r] : k1;      // first entry of row r
            bool head = rstart < k0;                       // row r began in an earlier segment
            // row ends: lane l of `win` holds the end of row rw + l, `ahead` the next 64 rows
            int32_t rw = r;
            int32_t win = row_end(row_ptr, n, static_cast<int64_t>(rw) + lane);
            int32_t ahead = row_end(row_ptr, n, static_cast<int64_t>(rw) + kWave + lane);
            // lanes l < kChunk: column index and weight of entry k + l of the coming round
            int32_t cw_col = 0;
            float cw_w = 0.0f;
            if (lane < kChunk && static_cast<int64_t>(k0) + lane < nnz) {
                cw_col = col[k0 + lane];
                cw_w = weight[k0 + lane];
            }
            double sum[kColPass];
#pragma unroll
            for (int j = 0; j < kColPass; ++j) sum[j] = 0.0;
            int32_t q0 = 0, qn = 0;   // rows q0 .. q0 + qn - 1 wait in the queue
            for (int32_t k = k0; k < k1;) {
                // (a) the rows that end in this round, at most kQueue: bit i of `ends` marks entry
                // k + i as the last of its row; the round stops at the kQueue-th end
                int32_t cnt = (k1 - k) < kChunk ? (k1 - k) : kChunk;
                uint32_t ends = 0;
                int32_t m = 0;
                for (int32_t rho = r;; ++rho) {
                    if (rho - rw == kWave) {
                        rw += kWave;
                        win = ahead;
                        ahead = row_end(row_ptr, n, static_cast<int64_t>(rw) + kWave + lane);
                    }
                    const int32_t e = lane_int(win, rho - rw);
                    if (e > k + cnt) break;
                    ends |= 1u << (e - 1 - k);
                    if (++m == kQueue) {
                        cnt = e - k;
                        break;
                    }
                }
                // (b) gather the round's rows of P (entries past the round repeat entry k)
                const int32_t cur_col = cw_col;
                const float cur_w = cw_w;
                float a[kChunk][kColPass];
#pragma unroll
                for (int j = 0; j < kColPass; ++j) {
                    // columns c0 + 64 j .. lie in block blk (uniform); each row's base is uniform
                    // and the lane adds its own offset
                    const int32_t blk = (c0 + j * kWave) / kWave;
                    const int64_t stride = p_block_width(blk, R);
                    const float* __restrict__ Pb = P32 + p_block_base(blk, n);
                    // lanes past column R - 1 read the row's first entry (their sums are never
                    // stored), so every load is issued unconditionally
                    const uint32_t off = c0 + lane + j * kWave < R ? static_cast<uint32_t>(lane) * 4u : 0u;
#pragma unroll
                    for (int i = 0; i < kChunk; ++i) {
                        const int32_t wi = lane_int(cur_col, i < cnt ? i : 0);
                        const char* row = reinterpret_cast<const char*>(Pb + static_cast<int64_t>(wi) * stride);
                        a[i][j] = *reinterpret_cast<const float*>(row + off);
                    }
                }
                // the next round's entries
                const int32_t kn = k + cnt;
                if (lane < kChunk && static_cast<int64_t>(kn) + lane < nnz) {
                    cw_col = col[kn + lane];
                    cw_w = weight[kn + lane];
                }
                // (c) finish the rows queued in the last round
                if (qn > 0) finish_queued(f, q0, qn, queue, pap);
                qn = 0;
                // (d) add the round's entries to their rows, in entry order
#pragma unroll
                for (int i = 0; i < kChunk; ++i) {
                    if (i < cnt) {
                    const double ti = static_cast<double>(lane_float(cur_w, i));
#pragma unroll
                    for (int j = 0; j < kColPass; ++j) sum[j] += ti * static_cast<double>(a[i][j]);
                    if ((ends >> i) & 1u) {   // row r ends at entry k + i
                        if (head) {
#pragma unroll
                            for (int j = 0; j < kColPass; ++j) {
                                const int32_t c = c0 + lane + j * kWave;
                                if (c < R) cut[(2 * wave) * R + c] = sum[j];
                            }
                            head = false;
                        } else {
                            if (qn == 0) q0 = r;
#pragma unroll
                            for (int j = 0; j < kColPass; ++j) queue[qn][lane + j * kWave] = sum[j];
                            ++qn;
                        }
#pragma unroll
                        for (int j = 0; j < kColPass; ++j) sum[j] = 0.0;
                        ++r;
                        rstart = k + i + 1;
                    }
                    }
                }
                k += cnt;
            }
            if (qn > 0) finish_queued(f, q0, qn, queue, pap);
            // the row open at the segment's end, cut by the boundary: its part to a slot
            if (head || rstart < k1) {
                const int64_t slot = 2 * wave + (head ? 0 : 1);
#pragma unroll
                for (int j = 0; j < kColPass; ++j) {
                    const int32_t c = c0 + lane + j * kWave;
                    if (c < R) cut[slot * R + c] = sum[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kColPass; ++j) {
            const int32_t c = c0 + lane + j * kWave;
            if (c < R) part[part_index(1, c, wave, R, nw)] = pap[j];
        }
    }
}

// The rows cut by segment boundaries.  Wave s (1 <= s < W) takes the row r holding entry
// seg_k[s] when r began in segment s - 1 (the first boundary inside r): its sum is the tail
// slot of s - 1 plus the head slots of s, s + 1, ... (every segment that starts inside r), in
// that order.  Its P.AP is added to the partial of wave s - 1, after that wave's own.
__global__ void spmm_fixup(int32_t n, int32_t v, int32_t R, int32_t W, const int32_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ seg_k, const int32_t* __restrict__ seg_row,
                           const double* __restrict__ d, const float* __restrict__ P32,
                           const double* __restrict__ cut, double* __restrict__ AP, double* __restrict__ part,
                           int32_t nw, const BpcgState* __restrict__ st) {
    if (st->ndone == R) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t s = 1 + (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave;
    if (s >= W) return;
    const int32_t r = seg_row[s];
    if (r >= n) return;
    const int32_t start = row_ptr[r];
    if (!(start < seg_k[s] && start >= seg_k[s - 1])) return;
    int64_t last = s;
    while (last + 1 < W && seg_row[last + 1] == r) ++last;
    const double du = d[r];
    for (int32_t c = lane; c < R; c += kWave) {
        double sum = cut[(2 * (s - 1) + 1) * R + c];
        for (int64_t q = s; q <= last; ++q) sum += cut[(2 * q) * R + c];
        const double p = static_cast<double>(P32[p_index(r, c, R, n)]);
        const double y = (r == v) ? 0.0 : du * p - sum;
        AP[static_cast<int64_t>(r) * R + c] = y;
        const int64_t i1 = part_index(1, c, s - 1, R, nw);
        part[i1] = part[i1] + p * y;
    }
}

// Waves of bpcg_spmm resident on the device at once, capped at kMaxWaves.
int64_t spmm_resident_waves() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bpcg_spmm, kBlock, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();   // the query's failure is not the caller's error
        per_cu = 4;
    }
    const int64_t w = static_cast<int64_t>(per_cu) * kWavesPerBlock * device_cu_count();
    return w < kMaxWaves ? w : kMaxWaves;
}

// X += alpha P, r -= alpha AP, and the partial dots z.r, z.r_old, r.r.  One thread per (row,
// column) element, rows strided, so every load and store is a contiguous stream; the thread
// count is a multiple of R, so thread t keeps column t mod R and its partials fill slot t
// (virtual wave t / R of the column-partial layout).
__global__ void bpcg_update(int32_t n, int32_t v, int32_t R, const ColScalars* __restrict__ sc,
                            const double* __restrict__ d, double* __restrict__ X, double* __restrict__ Rr,
                            const float* __restrict__ P32, const double* __restrict__ AP, double* __restrict__ part,
                            const BpcgState* __restrict__ st) {
    if (st->ndone == R) return;
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t rows_step = static_cast<int64_t>(gridDim.x) * blockDim.x / R;
    const int32_t c = static_cast<int32_t>(t % R);
    const double alpha = sc[c].alpha;
    double zr = 0.0, zro = 0.0, rr = 0.0;
    for (int64_t u = t / R; u < n; u += rows_step) {
        if (u == v) continue;
        const int64_t i = u * R + c;
        const double p = static_cast<double>(P32[p_index(u, c, R, n)]);
        X[i] = X[i] + alpha * p;
        const double r_old = Rr[i];
        const double r = r_old - alpha * AP[i];
        Rr[i] = r;
        const double z = r / d[u];
        zr += z * r;
        zro += z * r_old;
        rr += r * r;
    }
    const int64_t slot = t / R;
    part[part_index(0, c, slot, R, rows_step)] = zr;
    part[part_index(1, c, slot, R, rows_step)] = zro;
    part[part_index(2, c, slot, R, rows_step)] = rr;
}

// P = z + beta P (z = r / d), and the partial dot r.P with P as stored; element layout and
// partial slots as bpcg_update.
constexpr int kDirRows = 8;
__global__ void bpcg_direction(int32_t n, int32_t v, int32_t R, const ColScalars* __restrict__ sc,
                               const double* __restrict__ d, const double* __restrict__ Rr, float* __restrict__ P32,
                               double* __restrict__ rp_part, const BpcgState* __restrict__ st) {
    if (st->ndone == R) return;
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t rows_step = static_cast<int64_t>(gridDim.x) * blockDim.x / R;
    const int32_t c = static_cast<int32_t>(t % R);
    const double beta = sc[c].beta;
    double rp = 0.0;
    // kDirRows rows' loads in flight per thread (one row at a time leaves the kernel waiting on
    // memory latency); the dot keeps the row order
    int64_t u = t / R;
    for (; u + (kDirRows - 1) * rows_step < n; u += kDirRows * rows_step) {
        double r[kDirRows], du[kDirRows];
        float p_old[kDirRows];
#pragma unroll
        for (int q = 0; q < kDirRows; ++q) {
            const int64_t uq = u + q * rows_step;
            r[q] = Rr[uq * R + c];
            du[q] = d[uq];
            p_old[q] = P32[p_index(uq, c, R, n)];
        }
#pragma unroll
        for (int q = 0; q < kDirRows; ++q) {
            const int64_t uq = u + q * rows_step;
            if (uq == v) continue;
            const float p = static_cast<float>(r[q] / du[q] + beta * static_cast<double>(p_old[q]));
            P32[p_index(uq, c, R, n)] = p;
            rp += r[q] * static_cast<double>(p);
        }
    }
    for (; u < n; u += rows_step) {
        if (u == v) continue;
        const double r = Rr[u * R + c];
        const int64_t pi = p_index(u, c, R, n);
        const float p = static_cast<float>(r / d[u] + beta * static_cast<double>(P32[pi]));
        P32[pi] = p;
        rp += r * static_cast<double>(p);
    }
    rp_part[part_index(0, c, t / R, R, rows_step)] = rp;
}

// Sum of q[0 .. count) by the block's threads, thread t over t, t + kBlock, ... with
// kScalarBatch loads in flight (one at a time leaves the kernel waiting on memory latency once
// per partial); each thread's sum keeps the order of a plain strided loop.
__device__ double strided_sum(const double* __restrict__ q, int32_t count) {
    double a = 0.0;
    int32_t w = threadIdx.x;
    for (; w + (kScalarBatch - 1) * kBlock < count; w += kScalarBatch * kBlock) {
        double va[kScalarBatch];
#pragma unroll
        for (int j = 0; j < kScalarBatch; ++j) va[j] = q[w + j * kBlock];
#pragma unroll
        for (int j = 0; j < kScalarBatch; ++j) a += va[j];
    }
    for (; w < count; w += kBlock) a += q[w];
    return a;
}

// Per-column scalar steps; block c sums column c's partials (strided_sum, then a fixed tree
// over the threads).
//   mode 0: after init (zr, rr0 from `part`)
//   mode 1: after spmm (alpha = r.P / P.AP: r.P from `rp_part`, P.AP from `part`)
//   mode 2: after update (beta from z.r, z.r_old, r.r in `part`)
// `part` holds `nwaves` slots per value, `rp_part` `rp_slots`.
__global__ void bpcg_scalars(int32_t R, int32_t nwaves, const double* __restrict__ part, int32_t rp_slots,
                             const double* __restrict__ rp_part, ColScalars* sc, int mode, double tol2,
                             BpcgState* __restrict__ st) {
    __shared__ double la[kBlock], lb[kBlock], le[kBlock];
    const int32_t c = blockIdx.x;
    // every column done: the iteration is not run (ndone only grows, so the whole iteration
    // sees the same answer)
    if (mode != 0 && st->ndone == R) return;
    if (mode == 1 && c == 0 && threadIdx.x == 0) st->iters += 1;
    double a, b, e = 0.0;
    if (mode == 1) {
        a = strided_sum(rp_part + part_index(0, c, 0, R, rp_slots), rp_slots);
        b = strided_sum(part + part_index(1, c, 0, R, nwaves), nwaves);
    } else {
        a = strided_sum(part + part_index(0, c, 0, R, nwaves), nwaves);
        b = strided_sum(part + part_index(1, c, 0, R, nwaves), nwaves);
        if (mode == 2) e = strided_sum(part + part_index(2, c, 0, R, nwaves), nwaves);
    }
    la[threadIdx.x] = a;
    lb[threadIdx.x] = b;
    le[threadIdx.x] = e;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) {
            la[threadIdx.x] += la[threadIdx.x + h];
            lb[threadIdx.x] += lb[threadIdx.x + h];
            le[threadIdx.x] += le[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    a = la[0];
    b = lb[0];
    e = le[0];
    ColScalars s = sc[c];
    if (mode == 0) {
        s.zr = a;
        s.rr0 = b;
        s.rr = b;
        s.done = (b == 0.0) ? 1 : 0;
        s.alpha = 0.0;
        s.beta = 0.0;
        if (s.done) atomicAdd(&st->ndone, 1);
    } else if (mode == 1) {
        s.rp = a;
        s.pap = b;
        s.alpha = (s.done || b == 0.0) ? 0.0 : a / b;
    } else {
        s.rr = e;
        s.beta = (s.done || s.zr == 0.0) ? 0.0 : (a - b) / s.zr;
        s.zr = a;
        if (!s.done && e <= tol2 * s.rr0) {
            s.done = 1;
            atomicAdd(&st->ndone, 1);
        }
    }
    sc[c] = s;
}

// Sum of v over the kBlock threads of a block in a fixed tree order; every thread gets it.
__device__ double block_sum(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    const double total = lds[0];
    __syncthreads();
    return total;
}

// Column sums (for centring) in two fixed-order stages: block b sums its contiguous range of
// rows per column (threads over columns, so the reads are coalesced) into part[c nparts + b],
// then one block per column adds its nparts partials.
__global__ void column_partials(int32_t n, int32_t R, int32_t rows_per_block, const double* __restrict__ M,
                                double* __restrict__ part) {
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * rows_per_block;
    const int64_t hi = lo + rows_per_block < n ? lo + rows_per_block : n;
    for (int32_t c = threadIdx.x; c < R; c += blockDim.x) {
        double s = 0.0;
        for (int64_t u = lo; u < hi; ++u) s += M[u * R + c];
        part[static_cast<int64_t>(c) * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void column_finish(int32_t nparts, const double* __restrict__ part, double* __restrict__ out,
                              double scale) {
    __shared__ double lds[kBlock];
    const int32_t c = blockIdx.x;
    const double* q = part + static_cast<int64_t>(c) * nparts;
    double s = 0.0;
    for (int32_t b = threadIdx.x; b < nparts; b += kBlock) s += q[b];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[c] = s * scale;
}

__global__ void center_columns(int32_t n, int32_t R, const double* __restrict__ mean, double* __restrict__ M) {
    const int64_t total = static_cast<int64_t>(n) * R;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        M[i] = M[i] - mean[i % R];
}

struct EdgeScalars {
    double trgl;
    double dld;
};

// Over row ranges, one pair of partials per block: dLd = d^T B (column 1 of Z) and
// trGL^ = sum_i c_i y_i^T L^+ y_i, with the probe entries y recomputed from g (the solve has
// overwritten the right-hand sides).
__global__ void scalar_partials(int32_t n, int32_t R, int32_t rows_per_block, ProbeSpec ps,
                                const double* __restrict__ g, const int32_t* __restrict__ node_id,
                                const int32_t* __restrict__ rank, const double* __restrict__ coef,
                                const double* __restrict__ Z, const double* __restrict__ d,
                                double* __restrict__ part) {
    __shared__ double lds[kBlock];
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * rows_per_block;
    const int64_t hi = lo + rows_per_block < n ? lo + rows_per_block : n;
    double q = 0.0, t = 0.0;
    for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
        const double* zu = Z + u * R;
        q += d[u] * zu[1];
        const int32_t id = node_id[u];
        const double gu = g[id];
        if (gu == 0.0) continue;
        if (ps.k == 0) {
            const int32_t c = 2 + rank[id];
            t += coef[c] * (sqrt(fabs(gu)) * zu[c]);
        } else {
            const int32_t first = class_first_column(ps, gu);
            for (int32_t i = 0; i < ps.k; ++i)
                t += coef[first + i] * (probe_entry(ps, gu, static_cast<uint32_t>(id), i) * zu[first + i]);
        }
    }
    q = block_sum(q, lds);
    t = block_sum(t, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = q;
        part[2 * blockIdx.x + 1] = t;
    }
}

// dLd and trGL from the block partials (one block, fixed order).
__global__ void edge_scalars(int32_t nparts, const double* __restrict__ part, EdgeScalars* out) {
    __shared__ double lds[kBlock];
    double q = 0.0, t = 0.0;
    for (int32_t b = threadIdx.x; b < nparts; b += kBlock) {
        q += part[2 * b];
        t += part[2 * b + 1];
    }
    q = block_sum(q, lds);
    t = block_sum(t, lds);
    if (threadIdx.x == 0) {
        out->trgl = t;
        out->dld = q;
    }
}

// One thread per CSR entry (u, w) with u < w, i.e. per undirected edge; the row u of entry
// k is found by binary search, so hub rows spread over the whole grid.
constexpr int kEdgeCols = 16;
__global__ void edge_gradient(int32_t n, int64_t nnz, int32_t R, const int32_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ col, const int32_t* __restrict__ edge_id,
                              const double* __restrict__ Z, const double* __restrict__ coef,
                              const EdgeScalars* __restrict__ es, double G, double vol, double* __restrict__ grad) {
    const double trgl = es->trgl, dld = es->dld;
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < nnz;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t w = col[k];
        int32_t lo = 0, hi = n - 1;     // largest u with row_ptr[u] <= k
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (row_ptr[mid] <= k)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t u = lo;
        if (w < u) continue;
        const double* za = Z + u * R;
        const double* zb = Z + w * R;
        const double dA = za[0] - zb[0], sA = za[0] + zb[0];
        const double dB = za[1] - zb[1], sB = za[1] + zb[1];
        // kEdgeCols columns' loads in flight at a time (one pair at a time leaves the thread
        // waiting on memory once per column); q keeps the column order
        double q = 0.0;
        int32_t c = 2;
        for (; c + kEdgeCols <= R; c += kEdgeCols) {
            double a[kEdgeCols], b[kEdgeCols], f[kEdgeCols];
#pragma unroll
            for (int i = 0; i < kEdgeCols; ++i) {
                a[i] = za[c + i];
                b[i] = zb[c + i];
                f[i] = coef[c + i];
            }
#pragma unroll
            for (int i = 0; i < kEdgeCols; ++i) {
                const double t = a[i] - b[i];
                q += f[i] * (t * t);
            }
        }
        for (; c < R; ++c) {
            const double t = za[c] - zb[c];
            q += coef[c] * (t * t);
        }
        const double term_g = (2.0 * sB - dB * dB) / vol - (2.0 * dld) / (vol * vol);
        grad[edge_id[k]] = ((2.0 * trgl - vol * q) + (2.0 * dA * dB - 2.0 * sA)) + G * term_g;
    }
}

struct BwdLayout {
    WsHeader* header;
    double *Y, *X, *AP, *part, *rp_part, *cut, *colmean, *coef;
    float* P32;
    ColScalars* sc;
    BpcgState* bst;
    EdgeScalars* es;
    GPart* gpart;
    int32_t* gbase;
    int32_t* rank;
    int32_t *seg_k, *seg_row;
    size_t total;
};

constexpr int32_t kRowBlocks = 2048;   // blocks of the row-range passes over g

// The SpMM's head and tail slots are sized for the most segments the graph can be cut into.
BwdLayout carve_bwd(void* ws, int32_t n, int64_t nnz, int32_t R) {
    Carver c(ws);
    const size_t wmax = static_cast<size_t>(spmm_segments(nnz, n, kMaxWaves));
    BwdLayout L{};
    const size_t nr = static_cast<size_t>(n) * R;
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.Y = c.take<double>(nr);
    L.X = c.take<double>(nr);
    L.AP = c.take<double>(nr);
    L.P32 = c.take<float>(nr);
    L.part = c.take<double>(static_cast<size_t>(kMaxWaves) * R * 3);
    L.rp_part = c.take<double>(static_cast<size_t>(kDirSlots) * R);
    L.cut = c.take<double>(2 * wmax * R);
    L.colmean = c.take<double>(R);
    L.coef = c.take<double>(R);
    L.sc = c.take<ColScalars>(R);
    L.bst = c.take<BpcgState>(1);
    L.es = c.take<EdgeScalars>(1);
    L.gpart = c.take<GPart>(kRowBlocks);
    L.gbase = c.take<int32_t>(kRowBlocks);
    L.rank = c.take<int32_t>(n);
    L.seg_k = c.take<int32_t>(wmax + 1);
    L.seg_row = c.take<int32_t>(wmax + 1);
    L.total = c.used();
    return L;
}

// Bound of one adjoint call's solve columns (grid sizes and column indices stay in 32 bits).
constexpr int64_t kMaxSolveColumns = int64_t{1} << 24;

// Columns the workspace is sized for: sketch mode 2 + 2k (both sign classes); exact mode
// 2 + max_support.
int64_t workspace_columns(const rwc_backward_params* bp) {
    const int64_t k = bp->k;
    return 2 + (k > 0 ? 2 * k : static_cast<int64_t>(bp->max_support));
}

int check_params(const rwc_csr* g, const rwc_backward_params* bp) {
    if (!g || !bp) return fail(RWC_ERR_INVALID_ARG, "g and bp are required");
    if (g->n < 2) return fail(RWC_ERR_INVALID_ARG, "the graph has %d nodes", g->n);
    if (bp->k < 0) return fail(RWC_ERR_INVALID_ARG, "k must be >= 0");
    if (bp->k == 0 && (bp->max_support < 1 || bp->max_support > g->n))
        return fail(RWC_ERR_INVALID_ARG, "exact mode needs max_support in [1, n]");
    if (workspace_columns(bp) > kMaxSolveColumns)
        return fail(RWC_ERR_TOO_LARGE, "%lld solve columns (limit %lld)", static_cast<long long>(workspace_columns(bp)),
                    static_cast<long long>(kMaxSolveColumns));
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_backward_workspace(const rwc_csr* g, const rwc_backward_params* bp, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is required");
    RWC_CHECK(check_params(g, bp));
    *bytes = carve_bwd(nullptr, g->n, g->nnz, static_cast<int32_t>(workspace_columns(bp))).total;
    return RWC_OK;
}

extern "C" int rwc_backward(const rwc_csr* g, const double* grad_rwc, const rwc_backward_params* bp, double* grad_w,
                            int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!grad_rwc || !grad_w) return fail(RWC_ERR_INVALID_ARG, "grad_rwc and grad_w are required");
    RWC_CHECK(check_params(g, bp));
    RWC_CHECK(require_connected(g, "rwc_backward"));
    const int32_t n = g->n, v = g->pivot_index, k = bp->k;
    const int32_t Rmax = static_cast<int32_t>(workspace_columns(bp));
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_bwd(nullptr, n, g->nnz, Rmax).total));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double tol = bp->tol > 0 ? bp->tol : 1e-10;
    const int max_iter = bp->max_iter > 0 ? bp->max_iter : 20000;
    const int check = bp->check_every > 0 ? bp->check_every : 16;

    // 1. The support of g: counts per sign and the sum, per row block, read back once.  The
    // number of solve columns depends on them.
    BwdLayout L = carve_bwd(ws, n, g->nnz, Rmax);
    const int32_t rblocks = static_cast<int32_t>(blocks_for(n, 1) < kRowBlocks ? blocks_for(n, 1) : kRowBlocks);
    const int32_t rpb = static_cast<int32_t>((static_cast<int64_t>(n) + rblocks - 1) / rblocks);
    hipLaunchKernelGGL(header_start, dim3(1), dim3(1), 0, s, L.header);
    hipLaunchKernelGGL(g_partials, dim3(rblocks), dim3(kBlock), 0, s, n, rpb, grad_rwc, L.gpart);
    RWC_HIP(hipGetLastError());
    std::vector<GPart> gp(rblocks);
    RWC_HIP(hipMemcpyAsync(gp.data(), L.gpart, sizeof(GPart) * rblocks, hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    double G = 0.0;
    int64_t npos = 0, nneg = 0, nbad = 0;
    std::vector<int32_t> base(rblocks);
    int64_t nz = 0;
    for (int32_t b = 0; b < rblocks; ++b) {   // fixed order
        G += gp[b].sum;
        npos += gp[b].npos;
        nneg += gp[b].nneg;
        nbad += gp[b].nbad;
        base[b] = static_cast<int32_t>(nz);
        nz += gp[b].nnz;
    }
    if (nbad) return fail(RWC_ERR_INVALID_ARG, "grad_rwc holds %lld values that are not finite", (long long)nbad);
    if (nz == 0) {   // the loss is identically zero: so is its gradient
        hipLaunchKernelGGL(fill_zero, dim3(blocks_for(g->m, kBlock) < 8192 ? blocks_for(g->m, kBlock) : 8192),
                           dim3(kBlock), 0, s, grad_w, g->m);
        RWC_HIP(hipGetLastError());
        RWC_HIP(hipStreamSynchronize(s));
        if (iters) *iters = 0;
        return RWC_OK;
    }
    if (k == 0 && nz > bp->max_support)
        return fail(RWC_ERR_INVALID_ARG, "grad_rwc has %lld nonzeros, more than max_support = %d", (long long)nz,
                    bp->max_support);
    const int32_t R = static_cast<int32_t>(2 + (k == 0 ? nz : static_cast<int64_t>(k) * ((npos > 0) + (nneg > 0))));
    // the layout of this call (R columns) fits inside the workspace sized for Rmax
    L = carve_bwd(ws, n, g->nnz, R);
    ProbeSpec ps{k, npos > 0 ? 1 : 0, static_cast<uint32_t>(bp->seed), static_cast<uint32_t>(bp->seed >> 32)};
    std::vector<double> coef(R, 0.0);
    if (k > 0) {
        int32_t c = 2;
        for (int cls = 0; cls < 2; ++cls) {
            if ((cls == 0 ? npos : nneg) == 0) continue;
            for (int32_t i = 0; i < k; ++i) coef[c++] = (cls == 0 ? 1.0 : -1.0) / k;
        }
    }
    RWC_HIP(hipMemcpyAsync(L.coef, coef.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    RWC_HIP(hipMemcpyAsync(L.gbase, base.data(), sizeof(int32_t) * rblocks, hipMemcpyHostToDevice, s));
    // the host vectors above are read by the copies before the synchronisations below

    // 2. Right-hand sides, centred
    if (k == 0)
        hipLaunchKernelGGL(rank_nonzeros, dim3(rblocks), dim3(kBlock), 0, s, n, rpb, grad_rwc, L.gbase, L.rank, L.coef);
    const int64_t nr = static_cast<int64_t>(n) * R;
    const unsigned flat = blocks_for(nr, kBlock) < 8192 ? blocks_for(nr, kBlock) : 8192;
    hipLaunchKernelGGL(rhs_fill, dim3(flat), dim3(kBlock), 0, s, n, R, ps, grad_rwc, g->node_id, g->strength, L.rank,
                       L.Y);

    // one wave per row up to what the device holds at once; the SpMM's segments (one per wave,
    // the waves past them idle) fill every resident wave slot on large graphs, since the
    // gathers are bound by memory latency
    int64_t nwaves = n;
    if (nwaves > spmm_resident_waves()) nwaves = spmm_resident_waves();
    const unsigned wave_blocks = static_cast<unsigned>((nwaves + kWavesPerBlock - 1) / kWavesPerBlock);
    nwaves = static_cast<int64_t>(wave_blocks) * kWavesPerBlock;
    const int32_t nw = static_cast<int32_t>(nwaves);
    const int32_t rows_per_block = static_cast<int32_t>((static_cast<int64_t>(n) + wave_blocks - 1) / wave_blocks);
    // (the partial arrays hold kMaxWaves * R * 3 doubles >= wave_blocks * R)
    const int32_t nseg = spmm_segments(g->nnz, n, nwaves);
    const int32_t nnz = static_cast<int32_t>(g->nnz);
    hipLaunchKernelGGL(spmm_bounds, dim3(blocks_for(static_cast<int64_t>(nseg) + 1, kBlock)), dim3(kBlock), 0, s, n,
                       nnz, nseg, g->row_ptr, L.seg_k, L.seg_row);
    const unsigned fix_blocks = blocks_for(nseg > 1 ? nseg - 1 : 1, kWavesPerBlock);
    hipLaunchKernelGGL(column_partials, dim3(wave_blocks), dim3(kBlock), 0, s, n, R, rows_per_block, L.Y, L.part);
    hipLaunchKernelGGL(column_finish, dim3(R), dim3(kBlock), 0, s, static_cast<int32_t>(wave_blocks), L.part,
                       L.colmean, 1.0 / n);
    hipLaunchKernelGGL(center_columns, dim3(flat), dim3(kBlock), 0, s, n, R, L.colmean, L.Y);

    // 3. Batched PCG.  The update runs R * m blocks: m * kBlock rows in flight per column,
    // m * kBlock partial slots per column, m at most kUpdateSlots / kBlock (2048 slots per
    // column, R = 66: a gradient 5 % faster than with 8192 on BA(1e5, 4) and 1.4 % on R-MAT
    // scale 23, from fewer scattered partial writes and reads; 1024 slots are slower on both)
    const int64_t upd_m = blocks_for(n, kBlock) < kUpdateSlots / kBlock ? blocks_for(n, kBlock) : kUpdateSlots / kBlock;
    const unsigned upd_blocks = static_cast<unsigned>(upd_m * R);
    const int32_t upd_nw = static_cast<int32_t>(upd_m * kBlock);
    // bpcg_init and bpcg_direction (the r.P partials) on a grid of their own, same layout
    const int64_t dir_m = blocks_for(n, kBlock) < kDirSlots / kBlock ? blocks_for(n, kBlock) : kDirSlots / kBlock;
    const unsigned dir_blocks = static_cast<unsigned>(dir_m * R);
    const int32_t dir_nw = static_cast<int32_t>(dir_m * kBlock);
    const double tol2 = tol * tol;
    hipLaunchKernelGGL(bpcg_init, dim3(dir_blocks), dim3(kBlock), 0, s, n, v, R, g->strength, L.Y, L.X, L.P32,
                       L.part, L.rp_part, L.bst);
    hipLaunchKernelGGL(bpcg_scalars, dim3(R), dim3(kBlock), 0, s, R, dir_nw, L.part, dir_nw, L.rp_part, L.sc, 0,
                       tol2, L.bst);
    RWC_HIP(hipGetLastError());
    std::vector<ColScalars> host(R);
    BpcgState progress{};
    int it = 0;
    bool converged = false;
    while (!converged && it < max_iter) {
        const int chunk = (max_iter - it) < check ? (max_iter - it) : check;
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(bpcg_spmm, dim3(wave_blocks), dim3(kBlock), 0, s, n, v, R, nnz, nseg, g->row_ptr,
                               g->col, g->weight, g->strength, L.P32, L.seg_k, L.seg_row, L.AP, L.cut, L.part, L.bst);
            if (nseg > 1)
                hipLaunchKernelGGL(spmm_fixup, dim3(fix_blocks), dim3(kBlock), 0, s, n, v, R, nseg, g->row_ptr,
                                   L.seg_k, L.seg_row, g->strength, L.P32, L.cut, L.AP, L.part, nw, L.bst);
            hipLaunchKernelGGL(bpcg_scalars, dim3(R), dim3(kBlock), 0, s, R, nw, L.part, dir_nw, L.rp_part, L.sc, 1,
                               tol2, L.bst);
            hipLaunchKernelGGL(bpcg_update, dim3(upd_blocks), dim3(kBlock), 0, s, n, v, R, L.sc, g->strength, L.X,
                               L.Y, L.P32, L.AP, L.part, L.bst);
            hipLaunchKernelGGL(bpcg_scalars, dim3(R), dim3(kBlock), 0, s, R, upd_nw, L.part, dir_nw, L.rp_part, L.sc,
                               2, tol2, L.bst);
            hipLaunchKernelGGL(bpcg_direction, dim3(dir_blocks), dim3(kBlock), 0, s, n, v, R, L.sc, g->strength, L.Y,
                               L.P32, L.rp_part, L.bst);
        }
        RWC_HIP(hipGetLastError());
        it += chunk;
        RWC_HIP(hipMemcpyAsync(host.data(), L.sc, sizeof(ColScalars) * R, hipMemcpyDeviceToHost, s));
        RWC_HIP(hipMemcpyAsync(&progress, L.bst, sizeof(BpcgState), hipMemcpyDeviceToHost, s));
        RWC_HIP(hipStreamSynchronize(s));
        converged = true;
        for (int32_t c = 0; c < R; ++c) converged = converged && host[c].done;
    }
    // iterations run: the launches past the one where the last column converged return at once
    if (iters) *iters = progress.iters;
    if (!converged) {
        double worst = 0.0;
        for (int32_t c = 0; c < R; ++c)
            if (host[c].rr0 > 0) worst = std::fmax(worst, std::sqrt(host[c].rr / host[c].rr0));
        return fail(RWC_ERR_NOT_CONVERGED, "adjoint solves: worst relative residual %.3e after %d iterations", worst, it);
    }
    // 4. L^+ y = z - mean(z), the two scalars, and the per-edge gradient
    hipLaunchKernelGGL(column_partials, dim3(wave_blocks), dim3(kBlock), 0, s, n, R, rows_per_block, L.X, L.part);
    hipLaunchKernelGGL(column_finish, dim3(R), dim3(kBlock), 0, s, static_cast<int32_t>(wave_blocks), L.part,
                       L.colmean, 1.0 / n);
    hipLaunchKernelGGL(center_columns, dim3(flat), dim3(kBlock), 0, s, n, R, L.colmean, L.X);
    hipLaunchKernelGGL(scalar_partials, dim3(wave_blocks), dim3(kBlock), 0, s, n, R, rows_per_block, ps, grad_rwc,
                       g->node_id, L.rank, L.coef, L.X, g->strength, L.part);
    hipLaunchKernelGGL(edge_scalars, dim3(1), dim3(kBlock), 0, s, static_cast<int32_t>(wave_blocks), L.part, L.es);
    const unsigned edge_blocks = blocks_for(g->nnz, kBlock) < 16384 ? blocks_for(g->nnz, kBlock) : 16384;
    hipLaunchKernelGGL(edge_gradient, dim3(edge_blocks), dim3(kBlock), 0, s, n, g->nnz, R, g->row_ptr, g->col,
                       g->edge_id, L.X, L.coef, L.es, G, g->vol, grad_w);
    RWC_HIP(hipGetLastError());
    RWC_HIP(hipStreamSynchronize(s));
    return RWC_OK;
}
