// rwc_fastchol: FastChol (Section 4, Algorithm 2) on the GPU.
//
// 1. IChol(calL_v, delta) (Lemma 4.1): incomplete Cholesky of the grounded normalised Laplacian
//    with threshold dropping, left-looking, columns in ascending input id (the pivot v removed).
//    Column j starts as A(j:N, j) = (1, -w_xy / sqrt(d_x d_y) for the later neighbours) and
//    loses R(j, k) R(j:N, k) for every earlier column k with R(j, k) != 0, in ascending k; the
//    pivot is the square root of what is left on the diagonal, and an off-diagonal entry
//    x = w_i / pivot is kept when x != 0 and |x| >= delta * ||A(j:N, j)||_1 (the threshold
//    variant of MATLAB's ichol, which the paper's experiments use).
// 2. The windowed, sparsified inverse (Lemma 4.3 and Algorithm 2's loop), right to left:
//      S*(:, u) = e_u / R_uu - sum_{i in (u, u + w_u], R_iu != 0} (R_iu / R_uu) S~(:, i),
//    w_u = min(floor(w_s (1 + d_u / d_max)), N); a column of more than zeta nonzeros keeps the
//    shortest prefix, by decreasing magnitude (ties by row), whose dropped tail has 1-norm at
//    most eps_p ||S*(:, u)||_1; tau~_u = ||S~(:, u)||^2.
//
// Both recursions are chains: column j needs every earlier column its row reaches (IChol) and
// column u the later columns of its window with a factor entry (the inverse).  IChol has two
// forms with the same result:
//   - dense (the default while the matrix's packed lower triangle fits): right-looking on that
//     triangle in HBM; launch k forms column k + 1 of R on 16 workgroups while the others subtract
//     R(i, k) R(j, k) for step k's kept pairs, one launch per step;
//   - chain: left-looking on one wave, sparse throughout, for any size.
// The inverse's columns form a shallow dependency DAG, which eight waves of one workgroup run,
// each column on one wave with its lanes over the column's entries.
// Every floating-point operation happens in the order the serial algorithm performs it (each
// entry's updates in ascending k, norms and tails summed one entry at a time, sorts by total
// orders), so the factor, S~ and tau~ are the serial ones bit for bit.
#include <algorithm>

#include "common.hpp"
#include "device.hpp"

namespace rwc {
namespace {

constexpr int kSortCap = 4096;   // entries one column may hold while it is ordered in LDS

struct FcArgs {
    // the graph, in its internal order
    const int32_t* row_ptr;
    const int32_t* col;
    const float* weight;
    const double* strength;
    const int32_t* node_id;
    const int32_t* node_index;
    int32_t n;
    int32_t v;        // pivot, input id
    int32_t N;        // n - 1 columns
    int32_t zeta;
    double droptol, ws, eps_p;
    // factor R: column j is [r_ptr[j], r_ptr[j + 1]), diagonal first, rows ascending
    int64_t* r_ptr;
    int32_t* r_row;
    double* r_val;
    int64_t* r_colend;  // end of that column (r_ptr[column + 1]), so a row-list link needs no more
    int64_t* r_next;    // next entry of the same row (row lists in ascending column), -1 at the end
    int64_t* head;      // first and last entry of each row
    int64_t* tail;
    int64_t r_cap;
    // inverse S~: column u is s_len[u] entries from s_start[u], rows ascending
    int64_t* s_start;
    int32_t* s_len;
    int32_t* s_row;
    double* s_val;
    int64_t s_cap;
    // dense accumulators with stamps (entry i is live in column c when stamp[i] == c + 1)
    double* acc;
    int32_t* stamp;
    int32_t* touched;   // [N] the rows a column has reached, in the order reached (the inverse:
                        // acc, stamp and touched hold one slice of N per wave)
    int32_t* done;      // [N] the inverse: column published
    double* inv_val;    // the inverse: per wave, kSortCap entries to order a large column in
    int32_t* inv_row;
    double* dmax;
    double* dense;      // dense IChol: the lower triangle of S, packed by columns (column j holds
                        // rows j .. N - 1 from packed_column(j, N))
    double* colnorm;    // dense IChol: ||A(j:N, j)||_1 per column
    double* xk;         // dense IChol: R(i, j) of the last column j that kept row i ...
    int32_t* xstamp;    // ... and that j (-1 before any)
    int32_t* stage_row; // dense IChol, two columns by parity: each forming workgroup's kept
    double* stage_val;  // entries (rows ascending), stage_cap per workgroup ...
    uint32_t* stage_cnt;  // ... their counts [2][kFormGroups] ...
    double* stage_piv;    // ... the pivot [2] ...
    int32_t* stage_first; // ... and whether row j + 1 was kept [2]
    int64_t stage_cap;
    double* tau;        // [n] output by input id
    WsHeader* header;
    int64_t* counters;  // [2]: entries of R and of S~
};

// Words one lane writes and another reads later (the dense accumulator, its stamps and the row
// lists): relaxed atomics.  They are used only on memory that one wave alone touches (the chain's
// kernel is a single wave; each wave of the inverse has its own slices), so their scope is the
// wavefront, and so is the scope of wave_order(): a wave's vector memory operations are
// performed in the order it issues them, so ordering them needs no wait for the memory system,
// only that the compiler keep them in program order.
template <class T>
__device__ __forceinline__ T ld(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <class T>
__device__ __forceinline__ void st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void wave_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ int32_t node_of_column(int32_t j, int32_t v) { return j + (j >= v ? 1 : 0); }
__device__ __forceinline__ int32_t column_of_node(int32_t u, int32_t v) { return u - (u > v ? 1 : 0); }

// Lane l's value of x (l the same in every lane), exactly.
__device__ __forceinline__ double lane_value(double x, int l) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffull), l));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Lanes whose flag is set, in lane order: this lane's rank among them and their number.
__device__ __forceinline__ uint32_t rank_of(bool flag, uint32_t& count) {
    const uint64_t m = __ballot(flag);
    const int lane = threadIdx.x & (kWave - 1);
    count = static_cast<uint32_t>(__popcll(m));
    return static_cast<uint32_t>(__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (kWave - lane)))));
}

// Bitonic sort of len (<= kSortCap) entries, in LDS or in the wave's own global scratch, by one
// wave; less(a, b) a total order.
template <class Less>
__device__ void wave_sort(double* val, int32_t* row, int32_t len, Less less) {
    const int lane = threadIdx.x & (kWave - 1);
    int32_t size = 1;
    while (size < len) size <<= 1;
    for (int32_t i = len + lane; i < size; i += kWave) {   // padding sorts last
        val[i] = 0.0;
        row[i] = 0x7FFFFFFF;
    }
    wave_order();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the wave's LDS writes are done
    __builtin_amdgcn_wave_barrier();
    for (int32_t k = 2; k <= size; k <<= 1) {
        for (int32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int32_t i = lane; i < size; i += kWave) {
                const int32_t p = i ^ jj;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const bool pad_i = row[i] == 0x7FFFFFFF, pad_p = row[p] == 0x7FFFFFFF;
                    // padding is larger than any entry
                    const bool p_before_i = pad_i ? !pad_p : (!pad_p && less(val[p], row[p], val[i], row[i]));
                    if (p_before_i == up) {
                        const double tv = val[i];
                        val[i] = val[p];
                        val[p] = tv;
                        const int32_t tr = row[i];
                        row[i] = row[p];
                        row[p] = tr;
                    }
                }
            }
            wave_order();   // the buffers may be in global memory: keep the stages in order
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ void fill_i32(int32_t* p, int64_t count, int32_t value) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = value;
}

__global__ void __launch_bounds__(kWave) fc_begin(FcArgs A) {
    const int lane = threadIdx.x;
    if (lane == 0) {
        header_begin(A.header);
        A.counters[0] = 0;
        A.counters[1] = 0;
        A.r_ptr[0] = 0;
    }
    double m = 0.0;
    for (int32_t x = lane; x < A.n; x += kWave)
        if (A.node_id[x] != A.v) m = A.strength[x] > m ? A.strength[x] : m;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, kWave);
        m = o > m ? o : m;
    }
    if (lane == 0) *A.dmax = m;
    if (A.head) {   // the chain's row lists (absent for the dense factor)
        for (int64_t i = lane; i < A.N; i += kWave) {
            st(&A.head[i], int64_t{-1});
            st(&A.tail[i], int64_t{-1});
        }
    }
    for (int64_t u = lane; u < A.n; u += kWave) A.tau[u] = 0.0;
}

// One link of a row list in IChol's left-looking update: entry e = R(j, k), the next entry of
// row j, the end of column k, and kSpan entries of column k's suffix from some position p0 (lane
// l holds positions p0 + b kWave + l, clamped to written positions for the load).
constexpr int kBatch = 4;
constexpr int kSpan = kBatch * kWave;
struct Link {
    int64_t e, next, end;
    double rjk;
    int32_t row[kBatch];
    double val[kBatch];
};

__device__ __forceinline__ void load_span(const FcArgs& A, int64_t p0, int64_t rp, Link& L) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
        const int64_t p = p0 + b * kWave + lane;
        const int64_t pc = p < rp ? p : rp - 1;
        L.row[b] = A.r_row[pc];
        L.val[b] = A.r_val[pc];
    }
}

// Starts the loads of the link at e; e outside [0, rp) ends the list (L.e = -1).
__device__ __forceinline__ Link open_link(const FcArgs& A, int64_t e, int64_t rp) {
    Link L;
    if (e < 0 || e >= rp) {
        L.e = -1;
        return L;
    }
    L.e = e;
    L.next = ld(&A.r_next[e]);
    L.rjk = A.r_val[e];
    L.end = A.r_colend[e];
    load_span(A, e, rp, L);
    return L;
}

// acc[i] -= R(i, k) R(j, k) for the loaded span's rows i < L.end; rows reached for the first time
// in this column start from 0 and join the touched list.  The rows of one column are distinct,
// so the span's loads of stamps and accumulators all precede its stores.
__device__ __forceinline__ void update(const FcArgs& A, int64_t p0, const Link& L, int32_t stamp, uint32_t& nt) {
    const int lane = threadIdx.x;
    int32_t i[kBatch], sg[kBatch];
    double cur[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
        i[b] = p0 + b * kWave + lane < L.end ? L.row[b] : -1;
        const int32_t ic = i[b] >= 0 ? i[b] : L.row[0];   // a valid address for every lane
        sg[b] = ld(&A.stamp[ic]);
        cur[b] = ld(&A.acc[ic]);
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
        const bool fresh = i[b] >= 0 && sg[b] != stamp;
        uint32_t cnt = 0;
        const uint32_t r = rank_of(fresh, cnt);
        if (fresh) {
            st(&A.stamp[i[b]], stamp);
            st(&A.touched[nt + r], i[b]);   // distinct rows below N: nt never passes N
            cur[b] = 0.0;
        }
        nt += cnt;
        if (i[b] >= 0) st(&A.acc[i[b]], cur[b] - L.val[b] * L.rjk);
    }
    wave_order();
}

// IChol, one wave.
__global__ void __launch_bounds__(kWave) fc_ichol(FcArgs A) {
    __shared__ int32_t krow[kSortCap];   // the entries a column keeps, ordered by row here
    __shared__ double kval[kSortCap];
    int32_t* touched = A.touched;
    const int lane = threadIdx.x;
    const int32_t N = A.N, v = A.v;
    int64_t rp = 0;   // r_ptr[j], uniform
    for (int32_t j = 0; j < N; ++j) {
        const int32_t stamp = j + 1;
        const int32_t u = node_of_column(j, v);
        const int32_t x = A.node_index[u];
        const double du = A.strength[x];
        const int32_t beg = A.row_ptr[x], end = A.row_ptr[x + 1];
        // column j of A: the diagonal, then the later neighbours by ascending input id
        uint32_t nt = 0;
        if (lane == 0) {
            st(&A.acc[j], 1.0);
            st(&A.stamp[j], stamp);
            st(&touched[0], j);
        }
        nt = 1;
        double colnorm = 1.0;
        bool full = false;
        for (int32_t b0 = beg; b0 < end; b0 += kWave) {
            const int32_t k = b0 + lane;
            int32_t i = -1;
            double a = 0.0;
            if (k < end) {
                const int32_t y = A.col[k];
                const int32_t yid = A.node_id[y];
                if (yid > u && yid != v) {
                    i = column_of_node(yid, v);
                    a = -static_cast<double>(A.weight[k]) / sqrt(du * A.strength[y]);
                }
            }
            uint32_t cnt = 0;
            const uint32_t r = rank_of(i >= 0, cnt);
            if (i >= 0) {
                st(&A.acc[i], a);
                st(&A.stamp[i], stamp);
                st(&touched[nt + r], i);
            }
            nt += cnt;
            // the column's 1-norm, one entry at a time in row order
            for (int l = 0; l < kWave; ++l) {
                const double al = __shfl(a, l, kWave);
                const int32_t il = __shfl(i, l, kWave);
                if (il >= 0) colnorm += fabs(al);
            }
        }
        if (full) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        wave_order();
        // left-looking update: every earlier column k with R(j, k) != 0, ascending k (a row has
        // at most j entries left of the diagonal: the guard stops a corrupt list).  Pipelined by
        // one link: the next link's entry, its column end and the first kSpan entries of its
        // column suffix are loaded before this link's accumulator update, so a link costs about
        // one memory round trip (the accumulator's) instead of four.
        int64_t links = 0;
        Link cur = open_link(A, ld(&A.head[j]), rp);
        while (cur.e >= 0) {
            if (++links > j) {
                full = true;
                break;
            }
            const Link nxt = open_link(A, cur.next, rp);
            // a suffix longer than kSpan: each further span is loaded before the previous one
            // is applied
            for (int64_t p0 = cur.e;; p0 += kSpan) {
                const bool more = p0 + kSpan < cur.end;
                Link span = cur;
                if (more) load_span(A, p0 + kSpan, rp, span);
                update(A, p0, cur, stamp, nt);
                if (!more) break;
                cur = span;
            }
            cur = nxt;
        }
        if (full) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        wave_order();
        const double wjj = ld(&A.acc[j]);
        if (!(wjj > 0.0)) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrPivot));
            return;
        }
        const double piv = sqrt(wjj);
        // the drop rule over the reached rows, the survivors ordered by row in LDS, then
        // appended after the diagonal
        const double thr = A.droptol * colnorm;
        uint32_t kept = 0;
        for (uint32_t t0 = 0; t0 < nt && !full; t0 += kSpan) {
            int32_t i[kBatch];
            double xv[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const uint32_t t = t0 + b * kWave + lane;
                i[b] = t < nt ? ld(&touched[t < nt ? t : 0]) : -1;
            }
#pragma unroll
            for (int b = 0; b < kBatch; ++b) xv[b] = ld(&A.acc[i[b] >= 0 ? i[b] : j]);
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const double x = xv[b] / piv;
                const bool keep = i[b] >= 0 && i[b] != j && x != 0.0 && fabs(x) >= thr;
                uint32_t cnt = 0;
                const uint32_t r = rank_of(keep, cnt);
                if (kept + cnt > static_cast<uint32_t>(kSortCap)) {
                    full = true;
                    break;
                }
                if (keep) {
                    krow[kept + r] = i[b];
                    kval[kept + r] = x;
                }
                kept += cnt;
            }
        }
        if (full || rp + 1 + static_cast<int64_t>(kept) > A.r_cap) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        wave_sort(kval, krow, static_cast<int32_t>(kept),
                  [](double, int32_t ra, double, int32_t rb) { return ra < rb; });
        const int64_t colend = rp + 1 + static_cast<int64_t>(kept);
        if (lane == 0) {
            A.r_row[rp] = j;
            A.r_val[rp] = piv;
            A.r_colend[rp] = colend;
            st(&A.r_next[rp], int64_t{-1});
        }
        for (uint32_t t = lane; t < kept; t += kWave) {
            const int32_t i = krow[t];
            const int64_t pos = rp + 1 + t;
            A.r_row[pos] = i;
            A.r_val[pos] = kval[t];
            A.r_colend[pos] = colend;
            st(&A.r_next[pos], int64_t{-1});
            // append to row i's list (each lane a different row)
            const int64_t last = ld(&A.tail[i]);
            if (last < 0)
                st(&A.head[i], pos);
            else
                st(&A.r_next[last], pos);
            st(&A.tail[i], pos);
        }
        rp += 1 + kept;
        if (lane == 0) A.r_ptr[j + 1] = rp;
        wave_order();
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) A.counters[0] = rp;
}

// ---- IChol, dense right-looking ----
// S starts as the lower triangle of calL_v.  Step k takes column k of S after steps 0..k-1: its
// pivot and the entries that pass the drop rule become column k of R, and every kept pair
// i >= j loses R(i, k) R(j, k) from S(i, j).  Each S(i, j) meets its updates in ascending k, as
// in the left-looking chain, so the two forms give the same factor bit for bit.
//
// Launch k forms column k + 1 of R on kFormGroups workgroups, each over a contiguous range of its
// rows, into a staging area (two columns, by parity); the other workgroups apply step k's pairs,
// reading column k from the staging area, and one of them copies it, in row order, into the
// compact factor.
constexpr int kDenseBlock = 1024;
constexpr int kDenseWaves = kDenseBlock / kWave;
constexpr int kFormGroups = 16;   // workgroups forming a column
constexpr int kFormRows = 4;      // rows per thread in one round of a workgroup's range
constexpr int kDenseGrid = 256;   // workgroups of a launch
constexpr int kDenseItems = 4;    // (column, 64-row chunk) items a wave loads at once

// Offset of column j in the packed lower triangle of an N x N matrix (columns of N - j rows).
__host__ __device__ __forceinline__ int64_t packed_column(int64_t j, int64_t N) { return j * N - j * (j - 1) / 2; }

__global__ void fc_dense_clear(uint64_t* p, int64_t count) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// S = the lower triangle of calL_v (S must be zero), and colnorm[j] = ||A(j:N, j)||_1 summed down
// the column from the diagonal, as the chain sums it.  One wave per column.
__global__ void __launch_bounds__(256) fc_dense_scatter(FcArgs A) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t N = A.N, v = A.v;
    const int32_t waves = static_cast<int32_t>(blockDim.x / kWave);
    for (int32_t j = blockIdx.x * waves + threadIdx.x / kWave; j < N; j += gridDim.x * waves) {
        const int32_t u = node_of_column(j, v);
        const int32_t x = A.node_index[u];
        const double du = A.strength[x];
        const int32_t beg = A.row_ptr[x], end = A.row_ptr[x + 1];
        double* Sj = A.dense + (packed_column(j, N) - j);   // Sj[i], i >= j
        if (lane == 0) {
            Sj[j] = 1.0;
            A.xstamp[j] = -1;
        }
        double colnorm = 1.0;
        for (int32_t b0 = beg; b0 < end; b0 += kWave) {
            const int32_t k = b0 + lane;
            int32_t i = -1;
            double a = 0.0;
            if (k < end) {
                const int32_t y = A.col[k];
                const int32_t yid = A.node_id[y];
                if (yid > u && yid != v) {
                    i = column_of_node(yid, v);
                    a = -static_cast<double>(A.weight[k]) / sqrt(du * A.strength[y]);
                    Sj[i] = a;
                }
            }
            for (int l = 0; l < kWave; ++l) {
                const double al = __shfl(a, l, kWave);
                const int32_t il = __shfl(i, l, kWave);
                if (il >= 0) colnorm += fabs(al);
            }
        }
        if (lane == 0) A.colnorm[j] = colnorm;
    }
}

// Part p of column j of R.  Step j - 1's update of column j (the pairs (i, j) with R(j, j-1) != 0)
// is applied here, on the loaded values, and never stored: nothing reads column j of S
// afterwards.  xk/xstamp give R(i, j-1) by row.  The pivot is sqrt(S(j, j)); this workgroup's
// rows i (a contiguous range of j + 1 .. N - 1) whose x = S(i, j) / pivot is nonzero with
// |x| >= droptol colnorm[j] go, ascending, to its staging slots, and become xk/xstamp for column
// j + 1.  Rows are read q-major: round r, slot q, thread t reads row base + q * kDenseBlock + t.
__device__ void form_part(const FcArgs& A, int32_t j, int p, uint32_t* counts /* [kFormRows][kDenseWaves] */) {
    const int64_t N = A.N;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const double* Sj = A.dense + (packed_column(j, N) - j);   // Sj[i], i >= j
    const int64_t M = N - 1 - j;
    const int64_t R = (M + kFormGroups - 1) / kFormGroups;
    const int64_t lo = j + 1 + p * R;
    const int64_t hi = lo + R < N ? lo + R : N;
    const int par = j & 1;
    int32_t* srow = A.stage_row + (static_cast<int64_t>(par) * kFormGroups + p) * A.stage_cap;
    double* sval = A.stage_val + (static_cast<int64_t>(par) * kFormGroups + p) * A.stage_cap;
    double wjj = Sj[j];
    const int32_t xsj = A.xstamp[j];
    const double xkj = A.xk[j];
    const double thr = A.droptol * A.colnorm[j];
    const bool upd = j > 0 && xsj == j - 1;
    const double x0 = upd ? xkj : 0.0;   // R(j, j - 1), 0 when column j - 1 dropped row j
    if (upd) wjj = wjj - x0 * x0;
    const bool bad = !(wjj > 0.0);
    const double piv = sqrt(wjj);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    uint32_t kept = 0;
    bool first_kept = false;
    for (int64_t base = lo; base < hi; base += static_cast<int64_t>(kDenseBlock) * kFormRows) {
        double xv[kFormRows], xo[kFormRows];
        int32_t xs[kFormRows];
#pragma unroll
        for (int q = 0; q < kFormRows; ++q) {
            const int64_t i = base + q * kDenseBlock + threadIdx.x;
            const int64_t ic = i < hi ? i : j;   // a valid address for every thread
            xv[q] = Sj[ic];
            xs[q] = A.xstamp[ic];
            xo[q] = A.xk[ic];
        }
        if (bad) break;   // uniform
        uint64_t km[kFormRows];
#pragma unroll
        for (int q = 0; q < kFormRows; ++q) {
            const int64_t i = base + q * kDenseBlock + threadIdx.x;
            const double sv = upd && xs[q] == j - 1 ? xv[q] - xo[q] * x0 : xv[q];
            xv[q] = i < hi ? sv / piv : 0.0;
            const bool keep = i < hi && xv[q] != 0.0 && fabs(xv[q]) >= thr;
            if (i == j + 1) first_kept = keep;
            km[q] = __ballot(keep);
            if (lane == 0) counts[q * kDenseWaves + wave] = static_cast<uint32_t>(__popcll(km[q]));
        }
        __syncthreads();
        uint32_t at[kFormRows], round = 0;
#pragma unroll
        for (int q = 0; q < kFormRows; ++q) {
            uint32_t before = 0, all = 0;
            for (int w = 0; w < kDenseWaves; ++w) {
                const uint32_t c = counts[q * kDenseWaves + w];
                before += w < wave ? c : 0;
                all += c;
            }
            at[q] = kept + round + before;
            round += all;
        }
#pragma unroll
        for (int q = 0; q < kFormRows; ++q) {
            if ((km[q] >> lane) & 1ull) {
                const uint32_t pos = at[q] + static_cast<uint32_t>(__popcll(km[q] & below));
                const int32_t i = static_cast<int32_t>(base + q * kDenseBlock + threadIdx.x);
                srow[pos] = i;
                sval[pos] = xv[q];
                A.xk[i] = xv[q];   // this thread read row i's previous xk / xstamp above
                A.xstamp[i] = j;
            }
        }
        kept += round;
        __syncthreads();   // counts are rewritten by the next round
    }
    if (bad) {
        if (p == 0 && threadIdx.x == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrPivot));
        return;
    }
    if (threadIdx.x == 0) A.stage_cnt[par * kFormGroups + p] = kept;
    if (p == 0 && threadIdx.x == 0) {
        A.stage_piv[par] = piv;
        A.stage_first[par] = first_kept ? 1 : 0;   // thread 0 of part 0 holds row j + 1
    }
}

// The staged column k: entry a of its kept rows (ascending) from the parts' counts.
struct Staged {
    uint32_t pre[kFormGroups + 1];
    const int32_t* row;
    const double* val;
    int64_t cap;
    __device__ __forceinline__ int64_t slot(int32_t a) const {
        int p = 0;
#pragma unroll
        for (int q = 1; q < kFormGroups; ++q) p += static_cast<uint32_t>(a) >= pre[q] ? 1 : 0;
        return p * cap + (a - static_cast<int32_t>(pre[p]));
    }
};

// Launch k: workgroups 0 .. kFormGroups-1 form column k + 1; the others subtract R(i, k) R(j, k)
// from S(i, j) for the kept pairs of column k, except in column k + 1 (which the forming
// workgroups update as they read it), and the first of them copies column k into the factor.
__global__ void __launch_bounds__(kDenseBlock) fc_dense_step(FcArgs A, int32_t k) {
    __shared__ uint32_t counts[kFormRows * kDenseWaves];
    const int64_t N = A.N;
    // Forming a column reads no status (its barriers need every wave of the workgroup; after an
    // error it only fills the staging area, which nothing uses); the other workgroups, which
    // have no barriers, stop once an earlier launch or this one has reported one.
    if (blockIdx.x < kFormGroups) {
        if (k + 1 < N) form_part(A, k + 1, blockIdx.x, counts);
        return;
    }
    if (__hip_atomic_load(&A.header->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int par = k & 1;
    Staged st;
    st.pre[0] = 0;
#pragma unroll
    for (int q = 0; q < kFormGroups; ++q) st.pre[q + 1] = st.pre[q] + A.stage_cnt[par * kFormGroups + q];
    st.row = A.stage_row + static_cast<int64_t>(par) * kFormGroups * A.stage_cap;
    st.val = A.stage_val + static_cast<int64_t>(par) * kFormGroups * A.stage_cap;
    st.cap = A.stage_cap;
    const int32_t c = static_cast<int32_t>(st.pre[kFormGroups]);   // kept entries below the pivot
    if (blockIdx.x == kFormGroups) {
        // column k of the factor: the pivot, then the kept rows ascending
        const int64_t rp = A.r_ptr[k];
        if (rp + 1 + c > A.r_cap) {
            if (threadIdx.x == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        for (int32_t a = threadIdx.x; a < c; a += kDenseBlock) {
            const int64_t sl = st.slot(a);
            A.r_row[rp + 1 + a] = st.row[sl];
            A.r_val[rp + 1 + a] = st.val[sl];
        }
        if (threadIdx.x == 0) {
            A.r_row[rp] = k;
            A.r_val[rp] = A.stage_piv[par];
            A.r_ptr[k + 1] = rp + 1 + c;
            A.counters[0] = rp + 1 + c;
        }
    }
    const int32_t b_lo = A.stage_first[par];   // 1: row k + 1 was kept, column k + 1 is being formed
    // columns b = b_lo .. c-1 in items (h, b): rows a in [b + 64 h, min(b + 64 h + 64, c)).
    // Items are numbered h-major: chunk h has the c - b_lo - 64 h columns b < c - 64 h.
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t gw = static_cast<int64_t>(blockIdx.x - kFormGroups) * kDenseWaves + threadIdx.x / kWave;
    const int64_t nw = static_cast<int64_t>(gridDim.x - kFormGroups) * kDenseWaves;
    int64_t items = 0;
    for (int32_t h = 0; c - b_lo - 64 * h > 0; ++h) items += c - b_lo - 64 * h;
    for (int64_t t0 = gw; t0 < items; t0 += nw * kDenseItems) {
        int32_t ra[kDenseItems], rb[kDenseItems];
        double xa[kDenseItems], xb[kDenseItems], sv[kDenseItems];
        bool on[kDenseItems];
#pragma unroll
        for (int q = 0; q < kDenseItems; ++q) {
            int64_t t = t0 + q * nw;
            on[q] = false;
            ra[q] = rb[q] = 0;
            xa[q] = xb[q] = 0.0;
            if (t < items) {
                int32_t h = 0;
                while (t >= c - b_lo - 64 * h) {   // wave-uniform
                    t -= c - b_lo - 64 * h;
                    ++h;
                }
                const int32_t b = b_lo + static_cast<int32_t>(t);
                const int32_t a = b + 64 * h + lane;
                const int64_t sb = st.slot(b);
                rb[q] = st.row[sb];
                xb[q] = st.val[sb];
                if (a < c) {
                    const int64_t sa = st.slot(a);
                    on[q] = true;
                    ra[q] = st.row[sa];
                    xa[q] = st.val[sa];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kDenseItems; ++q)
            if (on[q]) sv[q] = A.dense[packed_column(rb[q], N) + (ra[q] - rb[q])];
#pragma unroll
        for (int q = 0; q < kDenseItems; ++q)
            if (on[q]) A.dense[packed_column(rb[q], N) + (ra[q] - rb[q])] = sv[q] - xa[q] * xb[q];
    }
}

// The windowed, sparsified inverse and tau~.  Column u needs exactly the later columns i of its
// window with R(i, u) != 0, which are few (0.9 on average on BA(20000, 5)), so the columns form a
// shallow DAG: kInvWaves waves of one workgroup take columns in descending order from a counter
// and each waits, on a done flag, for the columns it reads.  The wave holding the largest
// unfinished column never waits, so every wave finishes; a wait that outlasts kInvSpinLimit
// naps, or any error, stops the kernel.  Each wave has its own accumulator, stamps and touched
// list (a slice of N of each), and orders a column in LDS when it has at most kInvLds nonzeros,
// else in its own kSortCap-entry slice of global scratch.  A column's arithmetic is the serial
// one; only its place in the S~ pool depends on the schedule.
constexpr int kInvWaves = 8;
constexpr int kInvLds = 512;
constexpr int64_t kInvSpinLimit = int64_t{1} << 26;

__global__ void __launch_bounds__(kInvWaves * kWave) fc_inverse(FcArgs A) {
    __shared__ double lval[kInvWaves][kInvLds];
    __shared__ int32_t lrow[kInvWaves][kInvLds];
    __shared__ int32_t next_col;
    __shared__ unsigned long long pool;
    __shared__ int32_t abort_all;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int32_t N = A.N, v = A.v;
    if (threadIdx.x == 0) {
        next_col = 0;
        pool = 0;
        abort_all = A.header->status != 0 ? 1 : 0;   // the factor is incomplete
    }
    __syncthreads();
    const double dmax = *A.dmax;
    double* acc = A.acc + static_cast<int64_t>(wave) * N;
    int32_t* stamps = A.stamp + static_cast<int64_t>(wave) * N;
    int32_t* touched = A.touched + static_cast<int64_t>(wave) * N;
    // a wave stops on an error of its own or of another wave
    auto fail = [&](uint32_t code) {
        if (lane == 0) {
            atomicOr(&A.header->status, code);
            __hip_atomic_store(&abort_all, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    while (__hip_atomic_load(&abort_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
        int32_t t = 0;
        if (lane == 0) t = atomicAdd(&next_col, 1);
        t = __shfl(t, 0, kWave);
        if (t >= N) break;
        const int32_t u = N - 1 - t;
        const int32_t stamp = -(u + 1);   // negative stamps: the factor's are positive
        const int32_t node = node_of_column(u, v);
        const int32_t x = A.node_index[node];
        const int64_t c0 = A.r_ptr[u], c1 = A.r_ptr[u + 1];
        const double ruu = A.r_val[c0];
        int64_t w = static_cast<int64_t>(floor(A.ws * (1.0 + A.strength[x] / dmax)));
        if (w > N) w = N;
        uint32_t nt = 1;
        if (lane == 0) {
            st(&acc[u], 1.0 / ruu);
            st(&stamps[u], stamp);
            st(&touched[0], u);
        }
        wave_order();
        // the window's entries of column u, 64 at a time (lane l: entry p0 + l); their columns of
        // S~ are waited for together, then added in ascending row order, each a dependent load of
        // its entries and then of their stamps and accumulators
        bool stop = false;
        for (int64_t p0 = c0 + 1; p0 < c1 && !stop; p0 += kWave) {
            const int64_t p = p0 + lane;
            int32_t i = -1;
            double coef = 0.0;
            if (p < c1) {
                const int32_t r = A.r_row[p];
                if (r <= u + w) {
                    i = r;
                    coef = A.r_val[p] / ruu;
                }
            }
            const uint64_t live = __ballot(i >= 0);   // a prefix: rows ascend
            if (live == 0ull) break;
            int64_t spins = 0;
            while (__ballot(i >= 0 && __hip_atomic_load(&A.done[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) !=
                   0ull) {
                if (__hip_atomic_load(&abort_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0 ||
                    ++spins > kInvSpinLimit) {
                    stop = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (stop) break;
            int64_t s0 = 0;
            int32_t sl = 0;
            if (i >= 0) {
                s0 = A.s_start[i];
                sl = A.s_len[i];
            }
            for (uint64_t bits = live; bits != 0ull; bits &= bits - 1) {
                const int l = __builtin_ctzll(bits);
                const double cf = __shfl(coef, l, kWave);
                const int64_t b0 = __shfl(s0, l, kWave);
                const int32_t bl = __shfl(sl, l, kWave);
                for (int32_t q0 = 0; q0 < bl; q0 += kWave) {
                    const int32_t q = q0 + lane;
                    int32_t r = -1;
                    double sv = 0.0;
                    if (q < bl) {
                        r = A.s_row[b0 + q];
                        sv = A.s_val[b0 + q];
                    }
                    const int32_t rc = r >= 0 ? r : u;   // a valid address for every lane
                    const int32_t sg = ld(&stamps[rc]);
                    const double old = ld(&acc[rc]);
                    const bool fresh = r >= 0 && sg != stamp;
                    uint32_t cnt = 0;
                    const uint32_t rk = rank_of(fresh, cnt);
                    if (fresh) {
                        st(&stamps[r], stamp);
                        st(&touched[nt + rk], r);   // distinct rows below N
                    }
                    nt += cnt;
                    if (r >= 0) st(&acc[r], (fresh ? 0.0 : old) - cf * sv);
                }
                wave_order();
            }
        }
        if (stop) {
            if (__hip_atomic_load(&abort_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
                fail(static_cast<uint32_t>(kErrWait));   // a wait ran out (not expected)
            break;
        }
        wave_order();
        // the nonzeros of S*(:, u), in LDS when they fit, else in this wave's global scratch
        const bool small = nt <= static_cast<uint32_t>(kInvLds);
        double* val = small ? lval[wave] : A.inv_val + static_cast<int64_t>(wave) * kSortCap;
        int32_t* row = small ? lrow[wave] : A.inv_row + static_cast<int64_t>(wave) * kSortCap;
        uint32_t nz = 0;
        bool full = false;
        for (uint32_t t0 = 0; t0 < nt; t0 += kWave) {
            const uint32_t tt = t0 + lane;
            int32_t r = -1;
            double a = 0.0;
            if (tt < nt) {
                r = ld(&touched[tt]);
                a = ld(&acc[r]);
            }
            const bool live = r >= 0 && a != 0.0;
            uint32_t cnt = 0;
            const uint32_t rk = rank_of(live, cnt);
            if (nz + cnt > static_cast<uint32_t>(kSortCap)) {
                full = true;
                break;
            }
            if (live) {
                val[nz + rk] = a;
                row[nz + rk] = r;
            }
            nz += cnt;
        }
        if (full) {
            fail(static_cast<uint32_t>(kErrCapacity));
            break;
        }
        wave_order();
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        int32_t keep = static_cast<int32_t>(nz);
        if (static_cast<int64_t>(nz) > A.zeta) {
            wave_sort(val, row, static_cast<int32_t>(nz), [](double va, int32_t ra, double vb, int32_t rb) {
                const double a = fabs(va), b = fabs(vb);
                return a > b || (a == b && ra < rb);
            });
            // the 1-norm in sorted order, then the tail grown from the smallest entry: every lane
            // adds the same values in the same order, read from the lanes that loaded them
            double l1 = 0.0;
            for (int32_t t0 = 0; t0 < static_cast<int32_t>(nz); t0 += kWave) {
                const int32_t t = t0 + lane;
                const double a = t < static_cast<int32_t>(nz) ? fabs(val[t]) : 0.0;
                const int32_t m = static_cast<int32_t>(nz) - t0 < kWave ? static_cast<int32_t>(nz) - t0 : kWave;
                for (int32_t l = 0; l < m; ++l) l1 += lane_value(a, l);
            }
            const double lim = A.eps_p * l1;
            double tail = 0.0;
            int32_t k = static_cast<int32_t>(nz);
            for (bool more = true; more && k > 0;) {
                const int32_t base = k > kWave ? k - kWave : 0;   // entries [base, k), largest index first
                const int32_t t = base + lane;
                const double a = t < k ? fabs(val[t]) : 0.0;
                for (int32_t l = k - 1 - base; l >= 0; --l) {
                    const double x = lane_value(a, l);
                    if (!(tail + x <= lim)) {
                        more = false;
                        break;
                    }
                    tail += x;
                    --k;
                }
            }
            keep = k;
        }
        wave_sort(val, row, keep, [](double, int32_t ra, double, int32_t rb) { return ra < rb; });
        unsigned long long at = 0;
        if (lane == 0) at = atomicAdd(&pool, static_cast<unsigned long long>(keep));
        const int64_t sp = static_cast<int64_t>(__shfl(at, 0, kWave));
        if (sp + keep > A.s_cap) {
            fail(static_cast<uint32_t>(kErrCapacity));
            break;
        }
        for (int32_t k = lane; k < keep; k += kWave) {
            A.s_row[sp + k] = row[k];
            A.s_val[sp + k] = val[k];
        }
        double t2 = 0.0;   // ||S~(:, u)||^2 in row order, as above
        for (int32_t t0 = 0; t0 < keep; t0 += kWave) {
            const int32_t t = t0 + lane;
            const double a = t < keep ? val[t] : 0.0;
            const int32_t m = keep - t0 < kWave ? keep - t0 : kWave;
            for (int32_t l = 0; l < m; ++l) {
                const double x = lane_value(a, l);
                t2 += x * x;
            }
        }
        if (lane == 0) {
            A.s_start[u] = sp;
            A.s_len[u] = keep;
            A.tau[node] = t2;
        }
        // every lane's stores of column u are done before the flag that publishes it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) __hip_atomic_store(&A.done[u], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        wave_order();
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (threadIdx.x == 0 && abort_all == 0) A.counters[1] = static_cast<int64_t>(pool);
}

struct FcLayout {
    WsHeader* header;
    int64_t* counters;
    double* dmax;
    int64_t *r_ptr, *r_next, *r_colend, *head, *tail, *s_start;
    int32_t *r_row, *s_len, *s_row, *stamp, *touched, *done, *inv_row;
    double* inv_val;
    double *r_val, *s_val, *acc, *colnorm, *xk, *dense;
    int32_t* xstamp;
    int32_t* stage_row;
    double* stage_val;
    uint32_t* stage_cnt;
    double* stage_piv;
    int32_t* stage_first;
    int64_t stage_cap;
    size_t total;
};

// Dense IChol needs the (n - 1)(n) / 2 doubles of a packed triangle; the automatic choice takes
// it up to this many bytes (an eighth of the device's 288 GB: n - 1 <= 92681; BA(60000, 5)'s
// triangle factors 47x faster than the chain).
constexpr uint64_t kDenseAutoBytes = uint64_t{32} << 30;
constexpr int64_t kDenseMaxColumns = int64_t{1} << 20;

bool use_dense(const rwc_fastchol_params* p, int32_t n) {
    const uint64_t N = static_cast<uint64_t>(n - 1);
    if (p->method == RWC_FASTCHOL_DENSE) return true;
    if (p->method == RWC_FASTCHOL_CHAIN) return false;
    return N * (N + 1) / 2 * sizeof(double) <= kDenseAutoBytes;
}

FcLayout carve_fc(void* ws, int32_t n, int64_t r_cap, int64_t s_cap, bool dense) {
    Carver c(ws);
    FcLayout L{};
    const int64_t N = n - 1;
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.counters = c.take<int64_t>(2);
    L.dmax = c.take<double>(1);
    L.r_ptr = c.take<int64_t>(N + 1);
    L.s_start = c.take<int64_t>(N);
    L.s_len = c.take<int32_t>(N);
    L.stamp = c.take<int32_t>(kInvWaves * N);
    L.touched = c.take<int32_t>(kInvWaves * N);
    L.acc = c.take<double>(kInvWaves * N);
    L.done = c.take<int32_t>(N);
    L.inv_val = c.take<double>(kInvWaves * kSortCap);
    L.inv_row = c.take<int32_t>(kInvWaves * kSortCap);
    L.r_row = c.take<int32_t>(r_cap);
    L.r_val = c.take<double>(r_cap);
    L.s_row = c.take<int32_t>(s_cap);
    L.s_val = c.take<double>(s_cap);
    if (!dense) {   // the chain's row lists
        L.head = c.take<int64_t>(N);
        L.tail = c.take<int64_t>(N);
        L.r_next = c.take<int64_t>(r_cap);
        L.r_colend = c.take<int64_t>(r_cap);
    } else {
        L.colnorm = c.take<double>(N);
        L.xk = c.take<double>(N);
        L.xstamp = c.take<int32_t>(N);
        const size_t cap = static_cast<size_t>((N - 1 + kFormGroups - 1) / kFormGroups + 1);
        L.stage_row = c.take<int32_t>(2 * kFormGroups * cap);
        L.stage_val = c.take<double>(2 * kFormGroups * cap);
        L.stage_cnt = c.take<uint32_t>(2 * kFormGroups);
        L.stage_piv = c.take<double>(2);
        L.stage_first = c.take<int32_t>(2);
        L.stage_cap = static_cast<int64_t>(cap);
        L.dense = c.take<double>(static_cast<size_t>(N) * static_cast<size_t>(N + 1) / 2);
    }
    L.total = c.used();
    return L;
}

int check_fc(const rwc_csr* g, const rwc_fastchol_params* p) {
    if (!g || !p) return fail(RWC_ERR_INVALID_ARG, "g and p are required");
    if (g->n < 2 || !g->row_ptr || !g->node_id) return fail(RWC_ERR_INVALID_ARG, "g is not a built CSR");
    RWC_CHECK(require_connected(g, "rwc_fastchol"));
    if (!(p->droptol >= 0.0) || !(p->window >= 1.0) || p->zeta < 0 || !(p->eps_p >= 0.0))
        return fail(RWC_ERR_INVALID_ARG, "droptol and eps_p must be >= 0, window >= 1, zeta >= 0");
    if (p->factor_capacity < g->n - 1 || p->inverse_capacity < 0)
        return fail(RWC_ERR_INVALID_ARG, "factor_capacity must be at least n - 1 and inverse_capacity >= 0");
    if (p->method != RWC_FASTCHOL_AUTO && p->method != RWC_FASTCHOL_CHAIN && p->method != RWC_FASTCHOL_DENSE)
        return fail(RWC_ERR_INVALID_ARG, "method must be RWC_FASTCHOL_AUTO, _CHAIN or _DENSE");
    if (p->method == RWC_FASTCHOL_DENSE && g->n - 1 > kDenseMaxColumns)
        return fail(RWC_ERR_TOO_LARGE, "dense IChol takes at most %lld columns", static_cast<long long>(kDenseMaxColumns));
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_fastchol_workspace(const rwc_csr* g, const rwc_fastchol_params* p, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(check_fc(g, p));
    *bytes = carve_fc(nullptr, g->n, p->factor_capacity, p->inverse_capacity, use_dense(p, g->n)).total;
    return RWC_OK;
}

extern "C" int rwc_fastchol(const rwc_csr* g, const rwc_fastchol_params* p, double* tau, void* ws, size_t ws_bytes,
                            void* stream) {
    clear_error();
    RWC_CHECK(check_fc(g, p));
    if (!tau) return fail(RWC_ERR_INVALID_ARG, "tau is required");
    const bool dense = use_dense(p, g->n);
    RWC_CHECK(check_workspace(ws, ws_bytes,
                              carve_fc(nullptr, g->n, p->factor_capacity, p->inverse_capacity, dense).total));
    FcLayout L = carve_fc(ws, g->n, p->factor_capacity, p->inverse_capacity, dense);
    FcArgs A{};
    A.row_ptr = g->row_ptr;
    A.col = g->col;
    A.weight = g->weight;
    A.strength = g->strength;
    A.node_id = g->node_id;
    A.node_index = g->node_index;
    A.n = g->n;
    A.v = g->pivot;
    A.N = g->n - 1;
    A.zeta = p->zeta;
    A.droptol = p->droptol;
    A.ws = p->window;
    A.eps_p = p->eps_p;
    A.r_ptr = L.r_ptr;
    A.r_row = L.r_row;
    A.r_val = L.r_val;
    A.r_next = L.r_next;
    A.r_colend = L.r_colend;
    A.head = L.head;
    A.tail = L.tail;
    A.r_cap = p->factor_capacity;
    A.s_start = L.s_start;
    A.s_len = L.s_len;
    A.s_row = L.s_row;
    A.s_val = L.s_val;
    A.s_cap = p->inverse_capacity;
    A.acc = L.acc;
    A.stamp = L.stamp;
    A.touched = L.touched;
    A.done = L.done;
    A.inv_val = L.inv_val;
    A.inv_row = L.inv_row;
    A.dmax = L.dmax;
    A.dense = L.dense;
    A.colnorm = L.colnorm;
    A.xk = L.xk;
    A.xstamp = L.xstamp;
    A.stage_row = L.stage_row;
    A.stage_val = L.stage_val;
    A.stage_cnt = L.stage_cnt;
    A.stage_piv = L.stage_piv;
    A.stage_first = L.stage_first;
    A.stage_cap = L.stage_cap;
    A.tau = tau;
    A.header = L.header;
    A.counters = L.counters;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(fc_begin, dim3(1), dim3(kWave), 0, s, A);
    {
        const int64_t N = g->n - 1;
        hipLaunchKernelGGL(fill_i32, dim3(blocks_for(kInvWaves * N, 256)), dim3(256), 0, s, L.stamp, kInvWaves * N, 0);
        hipLaunchKernelGGL(fill_i32, dim3(blocks_for(N, 256)), dim3(256), 0, s, L.done, N, 0);
    }
    if (dense) {
        const int64_t N = g->n - 1;
        const int64_t cells = N * (N + 1) / 2;
        hipLaunchKernelGGL(fc_dense_clear, dim3(static_cast<unsigned>(std::min<int64_t>(blocks_for(cells, 256), 8192))),
                           dim3(256), 0, s, reinterpret_cast<uint64_t*>(L.dense), cells);
        hipLaunchKernelGGL(fc_dense_scatter, dim3(blocks_for(N, 256 / kWave)), dim3(256), 0, s, A);
        // one launch per step: launch k reads what every workgroup of launch k - 1 wrote; the
        // last one only copies column N - 1 into the factor
        for (int64_t k = -1; k < N; ++k)
            hipLaunchKernelGGL(fc_dense_step, dim3(k < 0 ? kFormGroups : kDenseGrid), dim3(kDenseBlock), 0, s, A,
                               static_cast<int32_t>(k));
    } else {
        hipLaunchKernelGGL(fc_ichol, dim3(1), dim3(kWave), 0, s, A);
    }
    hipLaunchKernelGGL(fc_inverse, dim3(1), dim3(kInvWaves * kWave), 0, s, A);
    RWC_HIP(hipGetLastError());
    return RWC_OK;
}

extern "C" int rwc_fastchol_sizes(const void* ws, int64_t* factor_entries, int64_t* inverse_entries, void* stream) {
    clear_error();
    if (!ws || !factor_entries || !inverse_entries) return fail(RWC_ERR_INVALID_ARG, "ws and outputs are required");
    FcLayout L = carve_fc(const_cast<void*>(ws), 2, 1, 0, false);
    int64_t c[2] = {0, 0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    RWC_HIP(hipMemcpyAsync(c, L.counters, sizeof(c), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    *factor_entries = c[0];
    *inverse_entries = c[1];
    return RWC_OK;
}
