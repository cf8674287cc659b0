// rwc_autotune_sampler: picks walkers per tree, trees in flight and (for walker teams) the
// schedule -- LDS path ring, shared or spread starts, ascending or breadth-first start order --
// for a graph by timing short probes of the real sampler, and caches the winner per graph class
// for the process.
//
// The sampler's outputs are a fixed function of (graph, seed, sample index), so the choice
// only changes speed.  Throughput depends on the number of concurrent walkers, on the state
// footprint they touch and on how the graph's walk lengths split across a team, which is why
// the choice is measured rather than derived.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace rwc {
namespace {

struct Candidate {
    int32_t W;
    int64_t T;
    uint32_t flags;   // schedule flags (0 = the automatic schedule)
};

using ClassKey = std::tuple<int, int, int, int>;  // log2 n, mean degree, weighted, log2 l

std::mutex g_mu;
std::map<ClassKey, rwc_tune_result> g_cache;

ClassKey class_of(const rwc_csr* g, int64_t l) {
    const int ln = static_cast<int>(std::floor(std::log2(static_cast<double>(g->n))));
    const int deg = static_cast<int>(std::lround(static_cast<double>(g->nnz) / g->n));
    const int ll = static_cast<int>(std::floor(std::log2(static_cast<double>(l))));
    return ClassKey{ln, deg, g->weighted, ll};
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Stage 1: one walker per tree with every tree in flight, and teams of 8 to 64 walkers with one
// or two device-fulls of resident waves or every tree in flight (the last avoids batch tails),
// all capped by the state budget, under the automatic schedule.
std::vector<Candidate> candidates(const rwc_csr* g, int64_t l, int64_t budget_bytes) {
    std::vector<Candidate> out;
    const int64_t stride = round_up(g->n, 8);
    const int64_t cap = budget_bytes / (8 * stride);
    auto add = [&](int W, int64_t T) {
        const int64_t S = 64 / W;
        if (T > l) T = l;
        T = round_up(T, S);
        if (T > cap) T = cap / S * S;
        if (T < S) return;
        for (const Candidate& c : out)
            if (c.W == W && c.T == T) return;
        out.push_back({W, T, 0u});
    };
    add(1, l);
    const int64_t resident = team_resident_waves(g->bfs_depth > 32);
    for (int W : {8, 16, 32, 64}) {
        const int64_t S = 64 / W;
        add(W, resident * S);
        add(W, 2 * resident * S);
        add(W, l);
    }
    return out;
}

// Stage 2, for a winning team: every combination of path ring, start sharing and start order.
std::vector<Candidate> schedules(const Candidate& best) {
    std::vector<Candidate> out;
    if (best.W == 1) return out;
    for (uint32_t ring : {RWC_SAMPLE_PATH_RING, RWC_SAMPLE_NO_PATH_RING})
        for (uint32_t share : {RWC_SAMPLE_SHARED_STARTS, RWC_SAMPLE_SPREAD_STARTS})
            for (uint32_t order : {RWC_SAMPLE_ID_STARTS, RWC_SAMPLE_BFS_STARTS})
                out.push_back({best.W, best.T, ring | share | order});
    return out;
}

struct TuneLayout {
    uint64_t* counts;
    uint64_t* steps;
    void* sample_ws;
    size_t sample_bytes;
    size_t total;
};

TuneLayout carve_tune(void* ws, const rwc_csr* g, size_t sample_bytes) {
    Carver c(ws);
    TuneLayout L{};
    L.counts = c.take<uint64_t>(g->n);
    L.steps = c.take<uint64_t>(1);
    L.sample_ws = c.take<char>(sample_bytes);
    L.sample_bytes = sample_bytes;
    L.total = c.used();
    return L;
}

int max_sample_bytes(const rwc_csr* g, const rwc_sample_params* p, const std::vector<Candidate>& cand,
                     size_t* bytes) {
    size_t best = 0;
    for (const Candidate& c : cand) {
        rwc_sample_params q = *p;
        q.walkers_per_tree = c.W;
        q.trees_in_flight = static_cast<int32_t>(c.T);
        q.num_samples = c.T;
        q.flags = c.flags;
        size_t b = 0;
        RWC_CHECK(rwc_sample_forests_workspace(g, 1, &q, &b));
        best = b > best ? b : best;
    }
    *bytes = best;
    return RWC_OK;
}

}  // namespace
}  // namespace rwc

using namespace rwc;

extern "C" int rwc_autotune_workspace(const rwc_csr* g, const rwc_sample_params* p, int64_t budget_bytes,
                                      size_t* bytes) {
    clear_error();
    if (!g || !p || !bytes || p->num_samples < 1 || budget_bytes <= 0)
        return fail(RWC_ERR_INVALID_ARG, "g, p and bytes are required; num_samples and budget must be positive");
    const std::vector<Candidate> cand = candidates(g, p->num_samples, budget_bytes);
    if (cand.empty()) return fail(RWC_ERR_WORKSPACE, "no candidate fits the state budget");
    size_t sb = 0;
    RWC_CHECK(max_sample_bytes(g, p, cand, &sb));
    *bytes = carve_tune(nullptr, g, sb).total;
    return RWC_OK;
}

extern "C" int rwc_autotune_sampler(const rwc_csr* g, const rwc_sample_params* p, int64_t budget_bytes,
                                    rwc_tune_result* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!g || !p || !out || p->num_samples < 1 || budget_bytes <= 0)
        return fail(RWC_ERR_INVALID_ARG, "g, p and out are required; num_samples and budget must be positive");
    const ClassKey key = class_of(g, p->num_samples);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *out = it->second;
            out->cached = 1;
            return RWC_OK;
        }
    }
    const std::vector<Candidate> cand = candidates(g, p->num_samples, budget_bytes);
    if (cand.empty()) return fail(RWC_ERR_WORKSPACE, "no candidate fits the state budget");
    size_t sb = 0;
    RWC_CHECK(max_sample_bytes(g, p, cand, &sb));
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_tune(nullptr, g, sb).total));
    TuneLayout L = carve_tune(ws, g, sb);
    rwc_tune_result best{};
    best.steps_per_s = -1.0;
    Candidate best_c = cand.front();
    auto probe = [&](const Candidate& c) -> int {
        rwc_sample_params q = *p;
        q.walkers_per_tree = c.W;
        q.trees_in_flight = static_cast<int32_t>(c.T);
        q.num_samples = c.T;        // one full batch of the real sample range
        q.flags = c.flags;
        float ms[2] = {0.f, 0.f};
        rwc_sample_outputs o{};
        o.counts = L.counts;
        o.total_steps = L.steps;
        o.timing_ms = ms;
        RWC_CHECK(rwc_sample_forests(g, 1, &q, &o, L.sample_ws, L.sample_bytes, stream));
        uint64_t steps = 0;
        RWC_HIP(hipMemcpy(&steps, L.steps, sizeof(steps), hipMemcpyDeviceToHost));
        const double rate = static_cast<double>(steps) / (1e-3 * (ms[0] + ms[1]));
        ++best.candidates;
        if (rate > best.steps_per_s) {
            best.steps_per_s = rate;
            best.walkers_per_tree = c.W;
            best.trees_in_flight = static_cast<int32_t>(c.T);
            best.flags = c.flags;
            best_c = c;
        }
        return RWC_OK;
    };
    for (const Candidate& c : cand) RWC_CHECK(probe(c));
    for (const Candidate& c : schedules(best_c)) RWC_CHECK(probe(c));
    best.cached = 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_cache[key] = best;
    }
    *out = best;
    return RWC_OK;
}

extern "C" void rwc_autotune_clear_cache(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
}
