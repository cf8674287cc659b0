/*
 * FastChol (Section 4, Algorithm 2), written as plainly as possible.
 *
 * TEST INFRASTRUCTURE ONLY (CPU oracle).  Shares no code with the HIP library.  Only the tests,
 * the package smoke check and the bench's CPU-baseline leg run it.
 *
 * Input: the grounded normalised Laplacian calL_v (node v removed) as its lower triangle in
 * compressed columns (column j holds rows i >= j, diagonal first, rows ascending).
 *
 * 1. IChol(calL_v, delta): incomplete Cholesky with threshold dropping, computed column by
 *    column (left-looking).  Column j starts as A(j:N, j); for every earlier column k with
 *    R(j, k) != 0, in ascending k, it loses R(j, k) R(j:N, k).  The pivot is the square root of
 *    the remaining diagonal; the other entries are divided by it and kept only when their
 *    magnitude is at least delta times the 1-norm of A(j:N, j) (the drop rule of the ICT
 *    variant of MATLAB's ichol, which the paper's experiments use; the diagonal is never
 *    dropped).
 * 2. The sparse approximate inverse S~ of R, column by column from the right (Lemma 4.3's
 *    recursion restricted to a window and sparsified):
 *      S*(:, u) = e_u / R_uu - sum_{i in (u, u + w_u], R_iu != 0} (R_iu / R_uu) S~(:, i),
 *    the products added in ascending i (entry by entry into a dense accumulator), with the
 *    window w_u = min(floor(w_s (1 + d_u / d_max)), N) from the base width w_s and u's degree.
 *    If S*(:, u) has at most zeta nonzeros it is kept whole; otherwise its entries are ordered by
 *    decreasing magnitude (ties by ascending row) and the shortest prefix is kept whose dropped
 *    tail has a 1-norm at most eps_p times the column's 1-norm (the tail summed from the
 *    smallest entry upwards).
 *    tau~_u = ||S~(:, u)||_2^2, summed in ascending row order.
 * tau~ estimates diag(calL_v^{-1}) and goes through the same assembly as FastWalk's t~.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* A growing array of (row, value) entries: the factor's columns are appended one after the
   other, column j occupying [ptr[j], ptr[j + 1]). */
typedef struct {
    int64_t len, cap;
    int64_t* row;
    double* val;
} entries_t;

static int entries_push(entries_t* e, int64_t r, double x) {
    if (e->len == e->cap) {
        const int64_t cap = e->cap ? 2 * e->cap : 1024;
        int64_t* nr = (int64_t*)realloc(e->row, (size_t)cap * sizeof(int64_t));
        if (!nr) return -2;
        e->row = nr;
        double* nv = (double*)realloc(e->val, (size_t)cap * sizeof(double));
        if (!nv) return -2;
        e->val = nv;
        e->cap = cap;
    }
    e->row[e->len] = r;
    e->val[e->len] = x;
    ++e->len;
    return 0;
}

/* Row lists: for each row i, the columns k < i with R(i, k) != 0 in the order they were made
   (ascending k) and the position of R(i, k) within the factor. */
typedef struct {
    int64_t len, cap;
    int64_t *next, *col, *pos;
} links_t;

static int links_push(links_t* l, int64_t* head, int64_t* tail, int64_t i, int64_t k, int64_t pos) {
    if (l->len == l->cap) {
        const int64_t cap = l->cap ? 2 * l->cap : 1024;
        int64_t* a = (int64_t*)realloc(l->next, (size_t)cap * sizeof(int64_t));
        if (!a) return -2;
        l->next = a;
        a = (int64_t*)realloc(l->col, (size_t)cap * sizeof(int64_t));
        if (!a) return -2;
        l->col = a;
        a = (int64_t*)realloc(l->pos, (size_t)cap * sizeof(int64_t));
        if (!a) return -2;
        l->pos = a;
        l->cap = cap;
    }
    const int64_t e = l->len++;
    l->next[e] = -1;
    l->col[e] = k;
    l->pos[e] = pos;
    if (tail[i] < 0)
        head[i] = e;
    else
        l->next[tail[i]] = e;
    tail[i] = e;
    return 0;
}

static int cmp_i64(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/*
 * IChol.  A: lower triangle of calL_v in CSC (a_ptr, a_row, a_val; rows ascending, the diagonal
 * first).  Returns 0 with the factor in r_ptr[N + 1] (caller's array) and *r_row / *r_val
 * (allocated here, released with oracle_free), -1 bad input, -2 out of memory, -3 a pivot <= 0.
 */
int oracle_ichol(int64_t N, const int64_t* a_ptr, const int64_t* a_row, const double* a_val, double droptol,
                 int64_t* r_ptr, int64_t** r_row, double** r_val, int64_t* r_nnz) {
    if (N < 1 || droptol < 0) return -1;
    entries_t R = {0, 0, NULL, NULL};
    links_t L = {0, 0, NULL, NULL, NULL};
    double* w = (double*)calloc((size_t)N, sizeof(double));
    unsigned char* mark = (unsigned char*)calloc((size_t)N, 1);
    int64_t* touched = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    int64_t* head = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    int64_t* tail = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    int rc = 0;
    if (!w || !mark || !touched || !head || !tail) {
        rc = -2;
        goto done;
    }
    for (int64_t i = 0; i < N; ++i) head[i] = tail[i] = -1;
    r_ptr[0] = 0;
    for (int64_t j = 0; j < N && rc == 0; ++j) {
        /* w = A(j:N, j) */
        int64_t nt = 0;
        double colnorm = 0.0;
        for (int64_t p = a_ptr[j]; p < a_ptr[j + 1]; ++p) {
            const int64_t i = a_row[p];
            if (i < j || i >= N) {
                rc = -1;
                break;
            }
            colnorm += fabs(a_val[p]);
            w[i] = a_val[p];
            mark[i] = 1;
            touched[nt++] = i;
        }
        if (rc) break;
        if (!mark[j]) {
            mark[j] = 1;
            touched[nt++] = j;
            w[j] = 0.0;
        }
        /* w -= R(j, k) R(j:N, k) for every earlier column k with R(j, k) != 0, ascending k */
        for (int64_t e = head[j]; e >= 0; e = L.next[e]) {
            const int64_t k = L.col[e];
            const double rjk = R.val[L.pos[e]];
            for (int64_t p = L.pos[e]; p < r_ptr[k + 1]; ++p) {   /* rows i >= j of column k */
                const int64_t i = R.row[p];
                if (!mark[i]) {
                    mark[i] = 1;
                    touched[nt++] = i;
                    w[i] = 0.0;
                }
                w[i] -= R.val[p] * rjk;
            }
        }
        if (!(w[j] > 0.0)) {
            rc = -3;
            break;
        }
        const double piv = sqrt(w[j]);
        qsort(touched, (size_t)nt, sizeof(int64_t), cmp_i64);
        if (entries_push(&R, j, piv)) {
            rc = -2;
            break;
        }
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t i = touched[t];
            if (i == j) continue;
            const double x = w[i] / piv;
            if (x != 0.0 && fabs(x) >= droptol * colnorm) {
                const int64_t pos = R.len;
                if (entries_push(&R, i, x) || links_push(&L, head, tail, i, j, pos)) {
                    rc = -2;
                    break;
                }
            }
        }
        r_ptr[j + 1] = R.len;
        for (int64_t t = 0; t < nt; ++t) {
            mark[touched[t]] = 0;
            w[touched[t]] = 0.0;
        }
    }
done:
    if (rc == 0) {
        *r_row = R.row;
        *r_val = R.val;
        *r_nnz = R.len;
    } else {
        free(R.row);
        free(R.val);
    }
    free(L.next);
    free(L.col);
    free(L.pos);
    free(w);
    free(mark);
    free(touched);
    free(head);
    free(tail);
    return rc;
}

void oracle_free(void* p) { free(p); }

typedef struct {
    int64_t row;
    double val;
} entry_t;

static int cmp_sparsify(const void* a, const void* b) {
    const entry_t* x = (const entry_t*)a;
    const entry_t* y = (const entry_t*)b;
    const double ax = fabs(x->val), ay = fabs(y->val);
    if (ax > ay) return -1;
    if (ax < ay) return 1;
    return (x->row > y->row) - (x->row < y->row);
}

static int cmp_row(const void* a, const void* b) {
    const entry_t* x = (const entry_t*)a;
    const entry_t* y = (const entry_t*)b;
    return (x->row > y->row) - (x->row < y->row);
}

/*
 * The sparse approximate inverse and tau~ (Algorithm 2's loop).  R: the IChol factor (CSC,
 * diagonal first in every column).  deg[N]: the degree d_u of each column's node, dmax their
 * maximum.  Writes tau[N] and, when s_nnz is given, the number of entries kept per column.
 * Returns 0, -1 bad input, -2 out of memory.
 */
static int sparse_inverse(int64_t N, const int64_t* r_ptr, const int64_t* r_row, const double* r_val,
                          const double* deg, double dmax, double ws, int64_t zeta, double eps_p, double* tau,
                          int64_t* s_nnz, int64_t dump_cap, int64_t* s_ptr, int64_t* s_row, double* s_val) {
    if (N < 1 || ws < 1 || zeta < 0 || eps_p < 0 || dmax <= 0) return -1;
    entry_t** S = (entry_t**)calloc((size_t)N, sizeof(entry_t*));
    int64_t* slen = (int64_t*)calloc((size_t)N, sizeof(int64_t));
    double* acc = (double*)calloc((size_t)N, sizeof(double));
    unsigned char* mark = (unsigned char*)calloc((size_t)N, 1);
    int64_t* touched = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    entry_t* col = (entry_t*)malloc((size_t)N * sizeof(entry_t));
    int rc = 0;
    if (!S || !slen || !acc || !mark || !touched || !col) { rc = -2; goto done; }
    for (int64_t u = N - 1; u >= 0 && rc == 0; --u) {
        const double ruu = r_val[r_ptr[u]];
        int64_t w = (int64_t)floor(ws * (1.0 + deg[u] / dmax));
        if (w > N) w = N;
        int64_t nt = 0;
        mark[u] = 1;
        touched[nt++] = u;
        acc[u] = 1.0 / ruu;
        for (int64_t p = r_ptr[u] + 1; p < r_ptr[u + 1]; ++p) {      /* rows i > u, ascending */
            const int64_t i = r_row[p];
            if (i > u + w) break;
            const double coef = r_val[p] / ruu;
            for (int64_t q = 0; q < slen[i]; ++q) {
                const int64_t r = S[i][q].row;
                if (!mark[r]) { mark[r] = 1; touched[nt++] = r; acc[r] = 0.0; }
                acc[r] -= coef * S[i][q].val;
            }
        }
        int64_t nz = 0;
        double l1 = 0.0;
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t r = touched[t];
            if (acc[r] != 0.0) {
                col[nz].row = r;
                col[nz].val = acc[r];
                ++nz;
            }
        }
        int64_t keep = nz;
        if (nz > zeta) {
            qsort(col, (size_t)nz, sizeof(entry_t), cmp_sparsify);
            for (int64_t t = 0; t < nz; ++t) l1 += fabs(col[t].val);
            /* smallest prefix whose dropped tail has 1-norm <= eps_p * l1: grow the tail from the
               smallest entry while it stays within the bound */
            double tail = 0.0;
            keep = nz;
            while (keep > 0 && tail + fabs(col[keep - 1].val) <= eps_p * l1) {
                tail += fabs(col[keep - 1].val);
                --keep;
            }
        }
        qsort(col, (size_t)keep, sizeof(entry_t), cmp_row);
        S[u] = (entry_t*)malloc((size_t)(keep > 0 ? keep : 1) * sizeof(entry_t));
        if (!S[u]) { rc = -2; break; }
        memcpy(S[u], col, (size_t)keep * sizeof(entry_t));
        slen[u] = keep;
        if (s_ptr) s_ptr[u] = keep;
        double t2 = 0.0;
        for (int64_t t = 0; t < keep; ++t) t2 += col[t].val * col[t].val;
        tau[u] = t2;
        if (s_nnz) s_nnz[u] = keep;
        for (int64_t t = 0; t < nt; ++t) { mark[touched[t]] = 0; acc[touched[t]] = 0.0; }
    }
    if (rc == 0 && s_ptr) {
        /* the kept columns as a CSC (s_ptr[N + 1], rows ascending within each column) */
        int64_t total = 0;
        for (int64_t u = 0; u < N; ++u) {
            const int64_t k = s_ptr[u];
            s_ptr[u] = total;
            total += k;
        }
        s_ptr[N] = total;
        if (total > dump_cap) {
            rc = -5;
        } else {
            for (int64_t u = 0; u < N; ++u)
                for (int64_t q = 0; q < slen[u]; ++q) {
                    s_row[s_ptr[u] + q] = S[u][q].row;
                    s_val[s_ptr[u] + q] = S[u][q].val;
                }
        }
    }
done:
    if (S)
        for (int64_t u = 0; u < N; ++u) free(S[u]);
    free(S); free(slen); free(acc); free(mark); free(touched); free(col);
    return rc;
}

int oracle_sparse_inverse(int64_t N, const int64_t* r_ptr, const int64_t* r_row, const double* r_val,
                          const double* deg, double dmax, double ws, int64_t zeta, double eps_p, double* tau,
                          int64_t* s_nnz) {
    return sparse_inverse(N, r_ptr, r_row, r_val, deg, dmax, ws, zeta, eps_p, tau, s_nnz, 0, NULL, NULL, NULL);
}

/* The same, also writing S~ as a CSC into caller arrays of capacity dump_cap (-5 if too small). */
int oracle_sparse_inverse_dump(int64_t N, const int64_t* r_ptr, const int64_t* r_row, const double* r_val,
                               const double* deg, double dmax, double ws, int64_t zeta, double eps_p, double* tau,
                               int64_t dump_cap, int64_t* s_ptr, int64_t* s_row, double* s_val) {
    return sparse_inverse(N, r_ptr, r_row, r_val, deg, dmax, ws, zeta, eps_p, tau, NULL, dump_cap, s_ptr, s_row,
                          s_val);
}
