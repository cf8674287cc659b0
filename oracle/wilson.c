/*
 * Serial FastWalk sampler (Section 5, Algorithm 3), written as plainly as possible.
 *
 * TEST INFRASTRUCTURE ONLY (CPU oracle).  Shares no code with the HIP library: this file
 * has its own Philox4x32-10, its own neighbour selection and its own counting.  Only the
 * tests, the package smoke check and the bench's CPU-baseline leg run it.
 *
 * For each sample i, one spanning tree rooted at the pivot (or a spanning forest rooted at a
 * root set) is grown by Wilson's loop-erased random walks.  The per-node count Algorithm 3
 * accumulates (+1 at the walk start, +1 at every arrival, -1 at the arrival that hits the
 * tree) equals the number of departures from the node, which is what is counted here.
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
 * One rooted spanning forest by Wilson's algorithm, written in terms of the quantity the
 * estimator needs: dep[u], the number of times the walk departs from u (Algorithm 3's visit
 * count of u: +1 at a walk start and at every arrival, -1 at the arrival that hits the tree,
 * is exactly the number of departures).
 *
 * in_tree starts as the root set.  Then every node j not yet in the tree, in the given order,
 * sends a random walk that records at each departure from u the arrow next[u] (overwriting
 * the arrows of erased loops) until it reaches the tree; the loop-erased path is then the
 * chain of arrows from j, which joins the tree.
 * Returns the number of RandomNeighbor calls, or UINT64_MAX when max_steps is exceeded.
 */
static uint64_t grow_forest(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                            uint64_t seed, uint32_t graph, uint64_t sample, const int32_t* order, uint64_t max_steps,
                            unsigned char* in_tree, int64_t* next, uint32_t* dep) {
    uint64_t calls = 0;
    for (int64_t jj = 0; jj < n; ++jj) {
        const int64_t j = order ? (int64_t)order[jj] : jj;
        /* the walk: one departure per step, the arrow of the latest departure kept */
        for (int64_t u = j; !in_tree[u]; u = next[u]) {
            next[u] = random_neighbor(u, dep[u], sample, graph, seed, row_ptr, col, cdf);
            dep[u] += 1;
            if (++calls > max_steps) return UINT64_MAX;
        }
        /* the loop-erased path from j joins the tree */
        for (int64_t u = j; !in_tree[u]; u = next[u]) in_tree[u] = 1;
    }
    return calls;
}

/*
 * Runs samples sample_begin .. sample_begin + nsamples - 1 of graph `graph`, each a spanning
 * forest rooted at the root set roots[0 .. nroots-1] (one root: a rooted spanning tree, the
 * case of Algorithm 3).
 *   visits     [n]        += per-node departure totals (Algorithm 3's t~ times l)
 *   visits_sq  [n]        += sum over samples of the squared per-sample departures (or NULL)
 *   steps      [nsamples]  = RandomNeighbor calls of each sample (or NULL)
 *   hash       [nsamples]  = sum over non-roots x of splitmix64(x * 2^32 + parent(x)) mod 2^64
 *   parents    [nsamples * n] parent of each node, -1 at the roots (or NULL)
 *   order      NULL for ascending node ids, else a permutation of 0..n-1
 * Returns 0, or -1 bad argument, -2 out of memory, -4 a sample needed more than max_steps
 * RandomNeighbor calls.
 */
int oracle_fastwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                    const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph, int64_t sample_begin,
                    int64_t nsamples, const int32_t* order, uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq,
                    uint64_t* steps, uint64_t* hash, int32_t* parents) {
    if (n < 1 || nroots < 1 || nroots >= n + 1 || nsamples < 0 || sample_begin < 0) return -1;
    for (int64_t r = 0; r < nroots; ++r)
        if (roots[r] < 0 || roots[r] >= n) return -1;
    unsigned char* is_root = (unsigned char*)calloc((size_t)n, 1);
    unsigned char* in_tree = (unsigned char*)malloc((size_t)n);
    int64_t* next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint32_t* dep = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    if (!is_root || !in_tree || !next || !dep) {
        free(is_root); free(in_tree); free(next); free(dep);
        return -2;
    }
    for (int64_t r = 0; r < nroots; ++r) is_root[roots[r]] = 1;
    int rc = 0;
    for (int64_t s = 0; s < nsamples && rc == 0; ++s) {
        const uint64_t sample = (uint64_t)(sample_begin + s);
        for (int64_t u = 0; u < n; ++u) {
            in_tree[u] = is_root[u];
            next[u] = -1;
            dep[u] = 0;
        }
        const uint64_t calls = grow_forest(n, row_ptr, col, cdf, seed, graph, sample, order, max_steps, in_tree,
                                           next, dep);
        if (calls == UINT64_MAX) {
            rc = -4;
            break;
        }
        uint64_t h = 0;
        for (int64_t u = 0; u < n; ++u) {
            visits[u] += (uint64_t)dep[u];
            if (visits_sq) visits_sq[u] += (uint64_t)dep[u] * (uint64_t)dep[u];
            if (!is_root[u]) h += splitmix64(((uint64_t)u << 32) | (uint64_t)(uint32_t)next[u]);
            if (parents) parents[s * n + u] = is_root[u] ? -1 : (int32_t)next[u];
        }
        if (steps) steps[s] = calls;
        if (hash) hash[s] = h;
    }
    free(is_root); free(in_tree); free(next); free(dep);
    return rc;
}

/*
 * The trap-walk estimator of (calL_v^{-1})_uu (Lemma 5.1 and the method the paper describes
 * after it): independent random walks from every node u != v that stop at the trap v, each
 * counting its visits to u (the start included).  The mean count estimates
 * t_u = (calL_v^{-1})_uu.
 *
 * Walk i from start node u takes its s-th step from the current node x by RandomNeighbor(x)
 * with the 64 random bits of Philox4x32-10 on the counter (s, u, i, graph ^ 2^31): one stream
 * per walk, its own graph word so that the walks never reuse a Wilson sample's draws.
 *   visits     [n]  += sum over the walks from u of their visit counts (0 at v)
 *   visits_sq  [n]  += sum of the squared counts (or NULL)
 *   steps           total RandomNeighbor calls (or NULL)
 * Walks i = walk_begin .. walk_begin + nwalks - 1 from every u != v.  Returns 0, -1 on a bad
 * argument, -4 if a walk exceeds max_steps.
 */
int oracle_trapwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf, int64_t v,
                    uint64_t seed, uint32_t graph, int64_t walk_begin, int64_t nwalks, uint64_t max_steps,
                    uint64_t* visits, uint64_t* visits_sq, uint64_t* steps) {
    if (n < 2 || v < 0 || v >= n || nwalks < 0 || walk_begin < 0) return -1;
    const uint32_t gword = graph ^ 0x80000000u;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t calls = 0;
    for (int64_t i = walk_begin; i < walk_begin + nwalks; ++i) {
        for (int64_t u = 0; u < n; ++u) {
            if (u == v) continue;
            uint64_t count = 1, s = 0;
            int64_t x = u;
            for (;;) {
                const uint32_t ctr[4] = {(uint32_t)s, (uint32_t)u, (uint32_t)i, gword};
                uint32_t o[4];
                oracle_philox4x32_10(ctr, key, o);
                const uint64_t r = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
                const int64_t beg = row_ptr[x], end = row_ptr[x + 1];
                int64_t pick;
                if (cdf == NULL) {
                    pick = (int64_t)(((u128)r * (u128)(uint64_t)(end - beg)) >> 64);
                } else {
                    const uint64_t target = (uint64_t)(((u128)r * (u128)cdf[end - 1]) >> 64);
                    pick = 0;
                    while (!(target < cdf[beg + pick])) ++pick;
                }
                x = col[beg + pick];
                ++s;
                if (s > max_steps) return -4;
                if (x == v) break;
                if (x == u) ++count;
            }
            calls += s;
            visits[u] += count;
            if (visits_sq) visits_sq[u] += count * count;
        }
    }
    if (steps) *steps += calls;
    return 0;
}
