/*
 * Serial FastWalk sampler: Algorithm 3 of the paper, written as plainly as possible.
 *
 * TEST INFRASTRUCTURE ONLY (CPU oracle).  Shares no code with the HIP library: this file
 * has its own Philox4x32-10, its own neighbour selection and its own counting.
 *
 * For each sample i, one spanning tree rooted at the pivot is grown by Wilson's algorithm
 * (Section 5): starting from every node in a fixed order, walk until the current tree is
 * hit, recording Next[u] at each departure, then retrace the loop-erased path from the
 * start marking it in the tree.  The visit vector follows Algorithm 3 exactly: +1 at the
 * walk start, +1 at every arrival, -1 at the arrival that hits the tree.
 *
 * RandomNeighbor(u) (Algorithm 3) is made reproducible by a counter-based generator:
 * the k-th departure from u in sample i of graph g uses Philox4x32-10 (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) on the counter
 * (k, u, i, g) with key (seed mod 2^32, seed >> 32).  Each node therefore owns a fixed
 * sequence of choices, which makes the sampled tree and all counts independent of the
 * order in which the walks are run (Wilson's cycle-popping argument); the optional
 * `order` argument exists so that tests can check that independence.
 *
 * Selection from the 64-bit word x = o0 + 2^32 o1:
 *   unweighted: k = floor(x * deg / 2^64);
 *   weighted:   r = floor(x * S / 2^64) with S the row total of the integer weights
 *               W_e = w_e * 2^24, and k the first position whose inclusive prefix sum of
 *               W exceeds r (a linear scan here).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- Philox4x32-10, from the round function and constants published in SC'11 ---- */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014) used as the tree checksum. */
static uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t z) { return splitmix64(z); }

static int64_t random_neighbor(int64_t u, uint32_t k, uint64_t sample, uint32_t graph, uint64_t seed,
                               const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf) {
    uint32_t ctr[4] = {k, (uint32_t)u, (uint32_t)sample, graph};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    oracle_philox4x32_10(ctr, key, o);
    const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    const int64_t beg = row_ptr[u], end = row_ptr[u + 1];
    const uint64_t deg = (uint64_t)(end - beg);
    int64_t pick;
    if (cdf == NULL) {
        pick = (int64_t)(((u128)x * (u128)deg) >> 64);
    } else {
        const uint64_t total = cdf[end - 1];
        const uint64_t r = (uint64_t)(((u128)x * (u128)total) >> 64);
        pick = 0;
        while (!(r < cdf[beg + pick])) ++pick;
    }
    return col[beg + pick];
}

/* RandomNeighbor on its own, exported so that tests can check the selection law. */
int64_t oracle_random_neighbor(int64_t u, uint32_t k, uint64_t sample, uint32_t graph, uint64_t seed,
                               const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf) {
    return random_neighbor(u, k, sample, graph, seed, row_ptr, col, cdf);
}

/*
 * Runs samples sample_begin .. sample_begin + nsamples - 1 of graph `graph`.
 *   visits     [n]        += per-node visit totals (Algorithm 3's t~ times l)
 *   visits_sq  [n]        += sum over samples of the squared per-sample visits (or NULL)
 *   steps      [nsamples]  = RandomNeighbor calls of each sample (or NULL)
 *   hash       [nsamples]  = sum_{x != root} splitmix64(x * 2^32 + parent(x)) mod 2^64 (or NULL)
 *   parents    [nsamples * n] parent of each node, -1 at the root (or NULL)
 *   order      NULL for ascending node ids, else a permutation of 0..n-1
 * Returns 0, or -1 bad argument, -2 out of memory, -3 visit/departure mismatch,
 * -4 a tree needed more than max_steps RandomNeighbor calls.
 */
int oracle_fastwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                    int64_t root, uint64_t seed, uint32_t graph, int64_t sample_begin, int64_t nsamples,
                    const int32_t* order, uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq,
                    uint64_t* steps, uint64_t* hash, int32_t* parents) {
    if (n < 1 || root < 0 || root >= n || nsamples < 0 || sample_begin < 0) return -1;
    unsigned char* in_tree = (unsigned char*)malloc((size_t)n);
    int64_t* next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* vis = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint32_t* departures = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    if (!in_tree || !next || !vis || !departures) {
        free(in_tree); free(next); free(vis); free(departures);
        return -2;
    }
    int rc = 0;
    for (int64_t s = 0; s < nsamples && rc == 0; ++s) {
        const uint64_t sample = (uint64_t)(sample_begin + s);
        for (int64_t u = 0; u < n; ++u) {
            in_tree[u] = 0;
            next[u] = -1;
            vis[u] = 0;
            departures[u] = 0;
        }
        in_tree[root] = 1;
        uint64_t calls = 0;
        for (int64_t jj = 0; jj < n && rc == 0; ++jj) {
            const int64_t j = order ? (int64_t)order[jj] : jj;
            if (j == root) continue;
            int64_t u = j;
            vis[u] += 1;
            while (!in_tree[u]) {
                next[u] = random_neighbor(u, departures[u], sample, graph, seed, row_ptr, col, cdf);
                departures[u] += 1;
                if (++calls > max_steps) { rc = -4; break; }
                u = next[u];
                vis[u] += 1;
            }
            if (rc) break;
            vis[u] -= 1;
            u = j;
            while (!in_tree[u]) {
                in_tree[u] = 1;
                u = next[u];
            }
        }
        if (rc) break;
        uint64_t h = 0;
        for (int64_t u = 0; u < n; ++u) {
            if ((uint64_t)vis[u] != (uint64_t)departures[u]) { rc = -3; break; }
            visits[u] += (uint64_t)vis[u];
            if (visits_sq) visits_sq[u] += (uint64_t)vis[u] * (uint64_t)vis[u];
            if (u != root) h += splitmix64(((uint64_t)u << 32) | (uint64_t)(uint32_t)next[u]);
            if (parents) parents[s * n + u] = (u == root) ? -1 : (int32_t)next[u];
        }
        if (steps) steps[s] = calls;
        if (hash) hash[s] = h;
    }
    free(in_tree); free(next); free(vis); free(departures);
    return rc;
}
