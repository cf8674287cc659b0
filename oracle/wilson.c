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

/*
 * Stratified stack entries (Latin hypercube sampling over the samples, McKay, Beckman and
 * Conover 1979).  With L = strata >= 2 and samples 0 .. L-1, the word of stack entry (u, k) in
 * sample i lies in stratum sigma(i) of [0, 2^64), where sigma is a permutation of 0 .. L-1
 * drawn for that entry alone:
 *   x     = the word above, from Philox on (k, u, i, g)
 *   a     = Philox4x32-10 on (k, u, 2^32 - 1, g)
 *   P     = a 4-round Feistel network on B = max(2, ceil(log2 L)) bits: the value is split
 *           into a high part of p = floor(B/2) bits and a low part of q = B - p bits; a round
 *           with key K maps (high, low) to (low, high xor (fmix32(low xor K) mod 2^p)) and
 *           the two widths trade places; keys a0, a1, a0 xor rotl(a1, 16), a1 xor rotl(a0, 16)
 *   pi(i) = P(i), P applied again while the result is >= L (cycle walking, a permutation)
 *   s     = floor(b * L / 2^64), b = a2 + 2^32 a3
 *   sigma = (pi(i) + s) mod L
 *   word  = sigma * M + floor(x * M / 2^64),  M = floor(2^64 / L)
 * For one sample the entries stay independent and (up to the 2^-64 grid) uniform, because
 * the shift s alone makes sigma(i) uniform; so every tree is still a Wilson tree.  Across the
 * L samples each entry visits every stratum once, which removes the additive part of the
 * variance of the mean count.  fmix32 is the 32-bit finaliser of MurmurHash3 (Appleby).
 */
static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

static uint64_t feistel4(uint64_t x, int bits, const uint32_t key[4]) {
    int p = bits / 2, q = bits - p;                 /* widths of the high and low parts */
    uint64_t high = x >> q, low = x & (((uint64_t)1 << q) - 1);
    for (int t = 0; t < 4; ++t) {
        const uint64_t f = (uint64_t)fmix32((uint32_t)low ^ key[t]) & (((uint64_t)1 << p) - 1);
        const uint64_t new_low = high ^ f;          /* p bits */
        high = low;                                 /* q bits */
        low = new_low;
        const int w = p;
        p = q;
        q = w;
    }
    return (high << q) | low;
}

/* The 64-bit word of the k-th departure from u in sample `sample` of graph `graph`. */
static uint64_t stack_word(uint32_t k, int64_t u, uint64_t sample, uint32_t graph, uint64_t seed, uint64_t strata) {
    uint32_t ctr[4] = {k, (uint32_t)u, (uint32_t)sample, graph};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    oracle_philox4x32_10(ctr, key, o);
    const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    if (strata < 2) return x;
    uint32_t a[4];
    ctr[2] = 0xFFFFFFFFu;
    oracle_philox4x32_10(ctr, key, a);
    const uint32_t round_keys[4] = {a[0], a[1], a[0] ^ rotl32(a[1], 16), a[1] ^ rotl32(a[0], 16)};
    int bits = 2;
    while (((uint64_t)1 << bits) < strata) ++bits;
    uint64_t y = sample;
    do {
        y = feistel4(y, bits, round_keys);
    } while (y >= strata);
    const uint64_t bw = (uint64_t)a[2] | ((uint64_t)a[3] << 32);
    const uint64_t shift = (uint64_t)(((u128)bw * (u128)strata) >> 64);
    const uint64_t stratum = (y + shift) % strata;
    const uint64_t width = (uint64_t)((((u128)1) << 64) / (u128)strata);
    return stratum * width + (uint64_t)(((u128)x * (u128)width) >> 64);
}

uint64_t oracle_stack_word(uint32_t k, int64_t u, uint64_t sample, uint32_t graph, uint64_t seed, uint64_t strata) {
    return stack_word(k, u, sample, graph, seed, strata);
}

static int64_t random_neighbor(int64_t u, uint32_t k, uint64_t sample, uint32_t graph, uint64_t seed,
                               uint64_t strata, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf) {
    const uint64_t x = stack_word(k, u, sample, graph, seed, strata);
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
    return random_neighbor(u, k, sample, graph, seed, 0, row_ptr, col, cdf);
}

int64_t oracle_random_neighbor_stratified(int64_t u, uint32_t k, uint64_t sample, uint32_t graph, uint64_t seed,
                                          uint64_t strata, const int64_t* row_ptr, const int32_t* col,
                                          const uint64_t* cdf) {
    return random_neighbor(u, k, sample, graph, seed, strata, row_ptr, col, cdf);
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
                            uint64_t seed, uint32_t graph, uint64_t sample, uint64_t strata, const int32_t* order,
                            uint64_t max_steps, unsigned char* in_tree, int64_t* next, uint32_t* dep) {
    uint64_t calls = 0;
    for (int64_t jj = 0; jj < n; ++jj) {
        const int64_t j = order ? (int64_t)order[jj] : jj;
        /* the walk: one departure per step, the arrow of the latest departure kept */
        for (int64_t u = j; !in_tree[u]; u = next[u]) {
            next[u] = random_neighbor(u, dep[u], sample, graph, seed, strata, row_ptr, col, cdf);
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
static int fastwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                    const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph, int64_t sample_begin,
                    int64_t nsamples, uint64_t strata, const int32_t* order, uint64_t max_steps, uint64_t* visits,
                    uint64_t* visits_sq, uint64_t* steps, uint64_t* hash, int32_t* parents) {
    if (n < 1 || nroots < 1 || nroots >= n + 1 || nsamples < 0 || sample_begin < 0) return -1;
    if (strata >= 2 && (strata > ((uint64_t)1 << 31) || (uint64_t)(sample_begin + nsamples) > strata)) return -1;
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
        const uint64_t calls = grow_forest(n, row_ptr, col, cdf, seed, graph, sample, strata, order, max_steps,
                                           in_tree, next, dep);
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

int oracle_fastwalk(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                    const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph, int64_t sample_begin,
                    int64_t nsamples, const int32_t* order, uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq,
                    uint64_t* steps, uint64_t* hash, int32_t* parents) {
    return fastwalk(n, row_ptr, col, cdf, roots, nroots, seed, graph, sample_begin, nsamples, 0, order, max_steps,
                    visits, visits_sq, steps, hash, parents);
}

/* The same with stratified stack entries over samples 0 .. strata - 1 (strata <= 2^31, the
 * run's samples inside that range; strata < 2 is the plain sampler). */
int oracle_fastwalk_stratified(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint64_t* cdf,
                               const int64_t* roots, int64_t nroots, uint64_t seed, uint32_t graph,
                               int64_t sample_begin, int64_t nsamples, uint64_t strata, const int32_t* order,
                               uint64_t max_steps, uint64_t* visits, uint64_t* visits_sq, uint64_t* steps,
                               uint64_t* hash, int32_t* parents) {
    return fastwalk(n, row_ptr, col, cdf, roots, nroots, seed, graph, sample_begin, nsamples, strata, order,
                    max_steps, visits, visits_sq, steps, hash, parents);
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
