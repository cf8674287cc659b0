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
        // trees in flight only shape HBM-state launches: stage 1 compares them in HBM
        out.push_back({W, T, W > 1 ? RWC_SAMPLE_NO_LDS_STATE : 0u});
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

// Stage 2, for a winning team: every combination of path ring, start sharing and start order,
// and for graphs whose trees fit in LDS, with the trees in LDS and in HBM.
std::vector<Candidate> schedules(const Candidate& best, bool lds_fits) {
    std::vector<Candidate> out;
    if (best.W == 1) return out;
    for (uint32_t lds : {0u, RWC_SAMPLE_NO_LDS_STATE}) {
        if (lds == 0 && !lds_fits) continue;
        for (uint32_t ring : {RWC_SAMPLE_PATH_RING, RWC_SAMPLE_NO_PATH_RING})
            for (uint32_t share : {RWC_SAMPLE_SHARED_STARTS, RWC_SAMPLE_SPREAD_STARTS})
                for (uint32_t order : {RWC_SAMPLE_ID_STARTS, RWC_SAMPLE_BFS_STARTS})
                    out.push_back({best.W, best.T, lds | ring | share | order});
    }
    return out;
}

// Whether a team of W walkers per tree keeps its trees in LDS on this graph (the sampler's rule
// for a single-graph call).
bool lds_fits(const rwc_csr* g, int W, int64_t l) {
    return W > 1 && (64 / W) * round_up(g->n, 8) * 8 <= 48 * 1024 && l <= (int64_t{1} << 24);
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
    RWC_CHECK(require_connected(g, "rwc_autotune_sampler"));
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
    for (const Candidate& c : schedules(best_c, lds_fits(g, best_c.W, best_c.T))) RWC_CHECK(probe(c));
    best.cached = 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_cache[key] = best;
    }
    *out = best;
    return RWC_OK;
}


// ---------------------------------------------------------------------------------------
// Multi-graph calls.
// ---------------------------------------------------------------------------------------
namespace rwc {
namespace {

struct BatchCandidate {
    int32_t w_mesh, w_other;
    uint32_t flags;
};

using BatchKey = std::tuple<int32_t, int64_t, int64_t, int64_t>;   // graphs, sum n, sum nnz, probe size
std::map<BatchKey, rwc_batch_tune_result> g_batch_cache;

int64_t probe_samples(int64_t l) {
    int64_t q = l / 8;
    if (q < 64) q = 64;
    return q < l ? q : l;
}

bool is_mesh(const rwc_csr& g) { return g.bfs_depth > 32; }

std::vector<BatchCandidate> batch_stage1() {
    std::vector<BatchCandidate> out;
    for (int wm : {16, 32, 64})
        for (int wo : {16, 32, 64}) out.push_back({wm, wo, 0u});
    return out;
}

std::vector<BatchCandidate> batch_stage2(const BatchCandidate& best) {
    std::vector<BatchCandidate> out;
    for (uint32_t lds : {0u, RWC_SAMPLE_NO_LDS_STATE})
        for (uint32_t ring : {RWC_SAMPLE_PATH_RING, RWC_SAMPLE_NO_PATH_RING})
            for (uint32_t order : {RWC_SAMPLE_ID_STARTS, RWC_SAMPLE_BFS_STARTS})
                out.push_back({best.w_mesh, best.w_other, lds | ring | order});
    return out;
}

struct BatchTuneLayout {
    uint64_t* counts;
    uint64_t* steps;
    void* sample_ws;
    size_t sample_bytes;
    size_t total;
};

BatchTuneLayout carve_batch_tune(void* ws, int64_t total_nodes, int32_t G, size_t sample_bytes) {
    Carver c(ws);
    BatchTuneLayout L{};
    L.counts = c.take<uint64_t>(total_nodes);
    L.steps = c.take<uint64_t>(G);
    L.sample_ws = c.take<char>(sample_bytes);
    L.sample_bytes = sample_bytes;
    L.total = c.used();
    return L;
}

rwc_sample_params batch_probe_params(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p,
                                     const BatchCandidate& c, std::vector<int32_t>& walkers) {
    walkers.resize(G);
    for (int32_t g = 0; g < G; ++g) walkers[g] = is_mesh(graphs[g]) ? c.w_mesh : c.w_other;
    rwc_sample_params q = *p;
    q.num_samples = probe_samples(p->num_samples);
    q.walkers_per_graph = walkers.data();
    q.walkers_per_tree = 0;
    q.trees_in_flight = 0;
    q.flags = (p->flags & (RWC_SAMPLE_PERSISTENT | RWC_SAMPLE_SHARED_STARTS | RWC_SAMPLE_SPREAD_STARTS)) | c.flags;
    q.flags |= RWC_SAMPLE_PERSISTENT;
    return q;
}

int batch_sample_bytes(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p, size_t* bytes) {
    size_t best = 0;
    std::vector<int32_t> walkers;
    std::vector<BatchCandidate> all = batch_stage1();
    for (const BatchCandidate& c : batch_stage1())
        for (const BatchCandidate& d : batch_stage2(c)) all.push_back(d);
    for (const BatchCandidate& c : all) {
        rwc_sample_params q = batch_probe_params(graphs, G, p, c, walkers);
        size_t b = 0;
        RWC_CHECK(rwc_sample_forests_workspace(graphs, G, &q, &b));
        best = b > best ? b : best;
    }
    *bytes = best;
    return RWC_OK;
}

int64_t sum_nodes(const rwc_csr* graphs, int32_t G) {
    int64_t t = 0;
    for (int32_t g = 0; g < G; ++g) t += graphs[g].n;
    return t;
}

}  // namespace
}  // namespace rwc

extern "C" int rwc_autotune_batch_workspace(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p,
                                            size_t* bytes) {
    clear_error();
    if (!graphs || !p || !bytes || G < 1 || p->num_samples < 1)
        return fail(RWC_ERR_INVALID_ARG, "graphs, p and bytes are required; num_graphs and num_samples must be positive");
    size_t sb = 0;
    RWC_CHECK(batch_sample_bytes(graphs, G, p, &sb));
    *bytes = carve_batch_tune(nullptr, sum_nodes(graphs, G), G, sb).total;
    return RWC_OK;
}

extern "C" int rwc_autotune_batch(const rwc_csr* graphs, int32_t G, const rwc_sample_params* p,
                                  rwc_batch_tune_result* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!graphs || !p || !out || G < 1 || p->num_samples < 1)
        return fail(RWC_ERR_INVALID_ARG, "graphs, p and out are required; num_graphs and num_samples must be positive");
    for (int32_t g = 0; g < G; ++g) RWC_CHECK(require_connected(&graphs[g], "rwc_autotune_batch"));
    int64_t nnz = 0;
    for (int32_t g = 0; g < G; ++g) nnz += graphs[g].nnz;
    const BatchKey key{G, sum_nodes(graphs, G), nnz, probe_samples(p->num_samples)};
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_batch_cache.find(key);
        if (it != g_batch_cache.end()) {
            *out = it->second;
            out->cached = 1;
            return RWC_OK;
        }
    }
    size_t sb = 0;
    RWC_CHECK(batch_sample_bytes(graphs, G, p, &sb));
    RWC_CHECK(check_workspace(ws, ws_bytes, carve_batch_tune(nullptr, sum_nodes(graphs, G), G, sb).total));
    BatchTuneLayout L = carve_batch_tune(ws, sum_nodes(graphs, G), G, sb);
    rwc_batch_tune_result best{};
    best.steps_per_s = -1.0;
    best.probe_samples = static_cast<int32_t>(probe_samples(p->num_samples));
    BatchCandidate best_c = batch_stage1().front();
    std::vector<int32_t> walkers;
    std::vector<uint64_t> steps(G);
    auto probe = [&](const BatchCandidate& c) -> int {
        rwc_sample_params q = batch_probe_params(graphs, G, p, c, walkers);
        float ms[2] = {0.f, 0.f};
        rwc_sample_outputs o{};
        o.counts = L.counts;
        o.total_steps = L.steps;
        o.timing_ms = ms;
        RWC_CHECK(rwc_sample_forests(graphs, G, &q, &o, L.sample_ws, L.sample_bytes, stream));
        RWC_HIP(hipMemcpy(steps.data(), L.steps, sizeof(uint64_t) * G, hipMemcpyDeviceToHost));
        uint64_t total = 0;
        for (uint64_t x : steps) total += x;
        const double rate = static_cast<double>(total) / (1e-3 * (ms[0] + ms[1]));
        ++best.candidates;
        if (rate > best.steps_per_s) {
            best.steps_per_s = rate;
            best.walkers_mesh = c.w_mesh;
            best.walkers_other = c.w_other;
            best.flags = c.flags;
            best_c = c;
        }
        return RWC_OK;
    };
    for (const BatchCandidate& c : batch_stage1()) RWC_CHECK(probe(c));
    for (const BatchCandidate& c : batch_stage2(best_c)) RWC_CHECK(probe(c));
    best.cached = 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_batch_cache[key] = best;
    }
    *out = best;
    return RWC_OK;
}

extern "C" void rwc_autotune_clear_cache(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
    g_batch_cache.clear();
}
