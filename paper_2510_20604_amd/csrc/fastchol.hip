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
// column u every later column in its window (the inverse).  One wave runs each chain column by
// column, its lanes over the column's entries.  Every floating-point operation happens in the
// order the serial algorithm performs it (updates in ascending k, norms and tails summed one
// entry at a time, sorts by total orders), so the factor, S~ and tau~ are the serial ones bit
// for bit.
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
    int32_t* r_colof;   // column of the entry at each position
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
    int32_t* touched;   // [N] the rows a column has reached, in the order reached
    double* dmax;
    double* tau;        // [n] output by input id
    WsHeader* header;
    int64_t* counters;  // [2]: entries of R and of S~
};

// Words one lane writes and another reads later (the dense accumulator, its stamps and the row
// lists): relaxed work-group-scope atomics, as for the walk kernels' tree state.
template <class T>
__device__ __forceinline__ T ld(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ void st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int32_t node_of_column(int32_t j, int32_t v) { return j + (j >= v ? 1 : 0); }
__device__ __forceinline__ int32_t column_of_node(int32_t u, int32_t v) { return u - (u > v ? 1 : 0); }

// Lanes whose flag is set, in lane order: this lane's rank among them and their number.
__device__ __forceinline__ uint32_t rank_of(bool flag, uint32_t& count) {
    const uint64_t m = __ballot(flag);
    const int lane = threadIdx.x & (kWave - 1);
    count = static_cast<uint32_t>(__popcll(m));
    return static_cast<uint32_t>(__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (kWave - lane)))));
}

// Bitonic sort of len (<= kSortCap) entries in LDS by one wave; less(a, b) a total order.
template <class Less>
__device__ void wave_sort(double* val, int32_t* row, int32_t len, Less less) {
    const int lane = threadIdx.x & (kWave - 1);
    int32_t size = 1;
    while (size < len) size <<= 1;
    for (int32_t i = len + lane; i < size; i += kWave) {   // padding sorts last
        val[i] = 0.0;
        row[i] = 0x7FFFFFFF;
    }
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
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
        }
    }
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
    for (int64_t i = lane; i < A.N; i += kWave) {
        st(&A.head[i], int64_t{-1});
        st(&A.tail[i], int64_t{-1});
        st(&A.stamp[i], 0);
    }
    for (int64_t u = lane; u < A.n; u += kWave) A.tau[u] = 0.0;
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
        __threadfence_block();
        // left-looking update: every earlier column k with R(j, k) != 0, ascending k (a row has
        // at most j entries left of the diagonal: the guard stops a corrupt list)
        int64_t links = 0;
        for (int64_t e = ld(&A.head[j]); e >= 0 && e < rp; e = ld(&A.r_next[e])) {
            if (++links > j) {
                full = true;
                break;
            }
            const int32_t k = A.r_colof[e];
            const double rjk = A.r_val[e];
            const int64_t kend = A.r_ptr[k + 1];
            for (int64_t p0 = e; p0 < kend; p0 += kWave) {
                const int64_t p = p0 + lane;
                int32_t i = -1;
                double rik = 0.0;
                bool fresh = false;
                if (p < kend) {
                    i = A.r_row[p];
                    rik = A.r_val[p];
                    fresh = ld(&A.stamp[i]) != stamp;
                }
                uint32_t cnt = 0;
                const uint32_t r = rank_of(fresh, cnt);
                double cur = 0.0;
                if (fresh) {
                    st(&A.stamp[i], stamp);
                    st(&touched[nt + r], i);   // distinct rows below N: nt never passes N
                } else if (i >= 0) {
                    cur = ld(&A.acc[i]);
                }
                nt += cnt;
                if (i >= 0) st(&A.acc[i], cur - rik * rjk);
            }
            __threadfence_block();
        }
        if (full) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        __threadfence_block();
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
        for (uint32_t t0 = 0; t0 < nt; t0 += kWave) {
            const uint32_t t = t0 + lane;
            int32_t i = -1;
            double xv = 0.0;
            if (t < nt) {
                i = ld(&touched[t]);
                if (i != j) xv = ld(&A.acc[i]) / piv;
            }
            const bool keep = i >= 0 && i != j && xv != 0.0 && fabs(xv) >= thr;
            uint32_t cnt = 0;
            const uint32_t r = rank_of(keep, cnt);
            if (kept + cnt > static_cast<uint32_t>(kSortCap)) {
                full = true;
                break;
            }
            if (keep) {
                krow[kept + r] = i;
                kval[kept + r] = xv;
            }
            kept += cnt;
        }
        if (full || rp + 1 + static_cast<int64_t>(kept) > A.r_cap) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        wave_sort(kval, krow, static_cast<int32_t>(kept),
                  [](double, int32_t ra, double, int32_t rb) { return ra < rb; });
        if (lane == 0) {
            A.r_row[rp] = j;
            A.r_val[rp] = piv;
            A.r_colof[rp] = j;
            st(&A.r_next[rp], int64_t{-1});
        }
        for (uint32_t t = lane; t < kept; t += kWave) {
            const int32_t i = krow[t];
            const int64_t pos = rp + 1 + t;
            A.r_row[pos] = i;
            A.r_val[pos] = kval[t];
            A.r_colof[pos] = j;
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
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) A.counters[0] = rp;
}

// The windowed, sparsified inverse and tau~, one wave, right to left.
__global__ void __launch_bounds__(kWave) fc_inverse(FcArgs A) {
    __shared__ double val[kSortCap];
    __shared__ int32_t row[kSortCap];
    __shared__ int32_t kept_count;
    int32_t* touched = A.touched;
    const int lane = threadIdx.x;
    const int32_t N = A.N, v = A.v;
    if (A.header->status != 0) return;   // the factor is incomplete
    const double dmax = *A.dmax;
    int64_t sp = 0;
    for (int32_t u = N - 1; u >= 0; --u) {
        const int32_t stamp = -(u + 1);   // negative stamps: the factor's are positive
        const int32_t node = node_of_column(u, v);
        const int32_t x = A.node_index[node];
        const int64_t c0 = A.r_ptr[u], c1 = A.r_ptr[u + 1];
        const double ruu = A.r_val[c0];
        int64_t w = static_cast<int64_t>(floor(A.ws * (1.0 + A.strength[x] / dmax)));
        if (w > N) w = N;
        uint32_t nt = 1;
        if (lane == 0) {
            st(&A.acc[u], 1.0 / ruu);
            st(&A.stamp[u], stamp);
            st(&touched[0], u);
        }
        __threadfence_block();
        bool full = false;
        for (int64_t p = c0 + 1; p < c1; ++p) {
            const int32_t i = A.r_row[p];
            if (i > u + w) break;
            const double coef = A.r_val[p] / ruu;
            const int64_t s0 = A.s_start[i];
            const int32_t sl = A.s_len[i];
            for (int32_t q0 = 0; q0 < sl; q0 += kWave) {
                const int32_t q = q0 + lane;
                int32_t r = -1;
                double sv = 0.0;
                bool fresh = false;
                if (q < sl) {
                    r = A.s_row[s0 + q];
                    sv = A.s_val[s0 + q];
                    fresh = ld(&A.stamp[r]) != stamp;
                }
                uint32_t cnt = 0;
                const uint32_t rk = rank_of(fresh, cnt);
                double cur = 0.0;
                if (fresh) {
                    st(&A.stamp[r], stamp);
                    st(&touched[nt + rk], r);   // distinct rows below N
                } else if (r >= 0) {
                    cur = ld(&A.acc[r]);
                }
                nt += cnt;
                if (r >= 0) st(&A.acc[r], cur - coef * sv);
            }
            __threadfence_block();
            if (full) break;
        }
        if (full) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        __threadfence_block();
        // the nonzeros of S*(:, u)
        uint32_t nz = 0;
        for (uint32_t t0 = 0; t0 < nt; t0 += kWave) {
            const uint32_t t = t0 + lane;
            int32_t r = -1;
            double a = 0.0;
            if (t < nt) {
                r = ld(&touched[t]);
                a = ld(&A.acc[r]);
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
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        int32_t keep = static_cast<int32_t>(nz);
        if (static_cast<int64_t>(nz) > A.zeta) {
            wave_sort(val, row, static_cast<int32_t>(nz), [](double va, int32_t ra, double vb, int32_t rb) {
                const double a = fabs(va), b = fabs(vb);
                return a > b || (a == b && ra < rb);
            });
            // the 1-norm in sorted order, then the tail grown from the smallest entry
            if (lane == 0) {
                double l1 = 0.0;
                for (int32_t t = 0; t < static_cast<int32_t>(nz); ++t) l1 += fabs(val[t]);
                double tail = 0.0;
                int32_t k = static_cast<int32_t>(nz);
                while (k > 0 && tail + fabs(val[k - 1]) <= A.eps_p * l1) {
                    tail += fabs(val[k - 1]);
                    --k;
                }
                kept_count = k;   // hand the count to the other lanes through LDS
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            keep = kept_count;
            __builtin_amdgcn_wave_barrier();
        }
        wave_sort(val, row, keep, [](double, int32_t ra, double, int32_t rb) { return ra < rb; });
        if (sp + keep > A.s_cap) {
            if (lane == 0) atomicOr(&A.header->status, static_cast<uint32_t>(kErrCapacity));
            return;
        }
        for (int32_t t = lane; t < keep; t += kWave) {
            A.s_row[sp + t] = row[t];
            A.s_val[sp + t] = val[t];
        }
        if (lane == 0) {
            double t2 = 0.0;
            for (int32_t t = 0; t < keep; ++t) t2 += val[t] * val[t];
            A.s_start[u] = sp;
            A.s_len[u] = keep;
            A.tau[node] = t2;
        }
        sp += keep;
        __threadfence_block();
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) A.counters[1] = sp;
}

struct FcLayout {
    WsHeader* header;
    int64_t* counters;
    double* dmax;
    int64_t *r_ptr, *r_next, *head, *tail, *s_start;
    int32_t *r_row, *r_colof, *s_len, *s_row, *stamp, *touched;
    double *r_val, *s_val, *acc;
    size_t total;
};

FcLayout carve_fc(void* ws, int32_t n, int64_t r_cap, int64_t s_cap) {
    Carver c(ws);
    FcLayout L{};
    const int64_t N = n - 1;
    L.header = c.take<WsHeader>(kHeaderBytes / sizeof(WsHeader));
    L.counters = c.take<int64_t>(2);
    L.dmax = c.take<double>(1);
    L.r_ptr = c.take<int64_t>(N + 1);
    L.head = c.take<int64_t>(N);
    L.tail = c.take<int64_t>(N);
    L.s_start = c.take<int64_t>(N);
    L.s_len = c.take<int32_t>(N);
    L.stamp = c.take<int32_t>(N);
    L.touched = c.take<int32_t>(N);
    L.acc = c.take<double>(N);
    L.r_row = c.take<int32_t>(r_cap);
    L.r_colof = c.take<int32_t>(r_cap);
    L.r_val = c.take<double>(r_cap);
    L.r_next = c.take<int64_t>(r_cap);
    L.s_row = c.take<int32_t>(s_cap);
    L.s_val = c.take<double>(s_cap);
    L.total = c.used();
    return L;
}

int check_fc(const rwc_csr* g, const rwc_fastchol_params* p) {
    if (!g || !p) return fail(RWC_ERR_INVALID_ARG, "g and p are required");
    if (g->n < 2 || !g->row_ptr || !g->node_id) return fail(RWC_ERR_INVALID_ARG, "g is not a built CSR");
    if (!(p->droptol >= 0.0) || !(p->window >= 1.0) || p->zeta < 0 || !(p->eps_p >= 0.0))
        return fail(RWC_ERR_INVALID_ARG, "droptol and eps_p must be >= 0, window >= 1, zeta >= 0");
    if (p->factor_capacity < g->n - 1 || p->inverse_capacity < 0)
        return fail(RWC_ERR_INVALID_ARG, "factor_capacity must be at least n - 1 and inverse_capacity >= 0");
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_fastchol_workspace(const rwc_csr* g, const rwc_fastchol_params* p, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(RWC_ERR_INVALID_ARG, "bytes is null");
    RWC_CHECK(check_fc(g, p));
    *bytes = carve_fc(nullptr, g->n, p->factor_capacity, p->inverse_capacity).total;
    return RWC_OK;
}

extern "C" int rwc_fastchol(const rwc_csr* g, const rwc_fastchol_params* p, double* tau, void* ws, size_t ws_bytes,
                            void* stream) {
    clear_error();
    RWC_CHECK(check_fc(g, p));
    if (!tau) return fail(RWC_ERR_INVALID_ARG, "tau is required");
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_fc(nullptr, g->n, p->factor_capacity, p->inverse_capacity).total));
    FcLayout L = carve_fc(ws, g->n, p->factor_capacity, p->inverse_capacity);
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
    A.r_colof = L.r_colof;
    A.r_next = L.r_next;
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
    A.dmax = L.dmax;
    A.tau = tau;
    A.header = L.header;
    A.counters = L.counters;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(fc_begin, dim3(1), dim3(kWave), 0, s, A);
    hipLaunchKernelGGL(fc_ichol, dim3(1), dim3(kWave), 0, s, A);
    hipLaunchKernelGGL(fc_inverse, dim3(1), dim3(kWave), 0, s, A);
    RWC_HIP(hipGetLastError());
    return RWC_OK;
}

extern "C" int rwc_fastchol_sizes(const void* ws, int64_t* factor_entries, int64_t* inverse_entries, void* stream) {
    clear_error();
    if (!ws || !factor_entries || !inverse_entries) return fail(RWC_ERR_INVALID_ARG, "ws and outputs are required");
    FcLayout L = carve_fc(const_cast<void*>(ws), 2, 1, 0);
    int64_t c[2] = {0, 0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    RWC_HIP(hipMemcpyAsync(c, L.counters, sizeof(c), hipMemcpyDeviceToHost, s));
    RWC_HIP(hipStreamSynchronize(s));
    *factor_entries = c[0];
    *inverse_entries = c[1];
    return RWC_OK;
}
