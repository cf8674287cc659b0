/* Runs the serial oracle (oracle/wilson.c) on small graphs so that a build with the address and
 * undefined-behaviour sanitizers can check its memory accesses and arithmetic: rooted trees and
 * root-set forests on a weighted and an unweighted graph, every output requested, stratified
 * stack entries, and the trap walks.  Exits 0 when every call returns 0. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fastwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                    const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph, int64_t sample_begin,
                    int64_t nsamples, const int32_t* order, uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq,
                    uint64_t* steps, uint64_t* hash, int32_t* parents);
int oracle_fastwalk_stratified(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                               const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph,
                               int64_t sample_begin, int64_t nsamples, uint64_t strata, const int32_t* order,
                               uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq, uint64_t* steps,
                               uint64_t* hash, int32_t* parents);
int oracle_trapwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf, int64_t v,
                    uint64_t seed, uint32_t graph, int64_t walk_begin, int64_t nwalks, uint64_t max_steps,
                    uint64_t* visits, uint64_t* visits_sq, uint64_t* steps);

/* a 6 x 6 grid, rows sorted by neighbour id, integer weights 2^24 (w = 1) and 3 * 2^24 */
enum { R = 6, N = R * R };

int main(void) {
    int64_t row_ptr[N + 1];
    int32_t col[4 * N];
    uint64_t cdf[4 * N];
    int64_t k = 0;
    for (int u = 0; u < N; ++u) {
        row_ptr[u] = k;
        const int r = u / R, c = u % R;
        const int nb[4] = {r > 0 ? u - R : -1, c > 0 ? u - 1 : -1, c < R - 1 ? u + 1 : -1, r < R - 1 ? u + R : -1};
        uint64_t run = 0;
        for (int i = 0; i < 4; ++i) {
            if (nb[i] < 0) continue;
            col[k] = nb[i];
            run += ((u + nb[i]) % 3 == 0 ? 3ull : 1ull) << 24;
            cdf[k] = run;
            ++k;
        }
    }
    row_ptr[N] = k;
    uint64_t visits[N] = {0}, visits_sq[N] = {0}, steps[8], hash[8];
    int32_t parents[8 * N];
    int32_t order[N];
    for (int i = 0; i < N; ++i) order[i] = (i * 7) % N;
    const int64_t one[1] = {14}, set[3] = {0, 20, 35};
    int rc = 0;
    rc |= oracle_fastwalk(N, row_ptr, col, NULL, one, 1, 5, 0, 0, 8, NULL, 1ull << 40, visits, visits_sq, steps, hash,
                          parents);
    rc |= oracle_fastwalk(N, row_ptr, col, cdf, set, 3, 6, 1, 3, 8, order, 1ull << 40, visits, visits_sq, steps, hash,
                          parents);
    rc |= oracle_fastwalk_stratified(N, row_ptr, col, cdf, one, 1, 9, 0, 5, 8, 13, NULL, 1ull << 40, visits,
                                     visits_sq, steps, hash, parents);
    rc |= oracle_fastwalk_stratified(N, row_ptr, col, NULL, set, 3, 10, 0, 0, 8, 1u << 31, order, 1ull << 40,
                                     visits, visits_sq, steps, hash, parents);
    uint64_t total = 0;
    rc |= oracle_trapwalk(N, row_ptr, col, cdf, 14, 7, 2, 0, 5, 1ull << 40, visits, visits_sq, &total);
    rc |= oracle_trapwalk(N, row_ptr, col, NULL, 0, 8, 2, 4, 3, 1ull << 40, visits, NULL, &total);
    printf("rc=%d steps=%llu\n", rc, (unsigned long long)total);
    return rc == 0 ? 0 : 1;
}
