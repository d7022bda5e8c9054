// Schedule autotuner (include/hgm.h, hgm_tune*): picks the schedule fields of
// hgm_opts (launch shapes, hub and solo bounds, clear form, first batch of
// rounds) for one instance or one batch by timing whole matchings on the
// device, and keeps the result in a text cache keyed by device and shape
// bucket so that later calls of the same shape reuse it.
//
// Every schedule computes the same bitmap (the matching is determined by the
// instance, the seed and the priority rule); the tuner checks that on every
// candidate it times, against the bitmap of the starting schedule, and
// reports a mismatch instead of choosing that candidate.
//
// Search: coordinate descent in a fixed order of fields, each over a short
// list of candidate values around the default, keeping a value only when it
// is faster than the best so far by more than the run-to-run spread (2%).
// Time of a candidate = median over `reps` calls of the host wall time of
// hgm_match / hgm_match_batch (which returns once the matching is complete
// in device memory), after one untimed call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "hgm.h"
#include "schedule.h"

namespace {

using namespace hgm;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Knob {
    const char *name;
    int32_t hgm_opts::*field;
    std::vector<int32_t> values;  // candidates (0 = library default)
    int kind;                     // 0: both, 1: batches only, 2: one instance only
};

std::vector<Knob> knobs(bool batch) {
    std::vector<Knob> k = {
        {"solo", &hgm_opts::solo_max_kappa, {-1, 1 << 16, 1 << 18, 1 << 20, 1 << 22}, 1},
        {"grid", &hgm_opts::edge_grid, {512, 1024, 1536, 2048, 3072, 4096, 8192, 16384}, 0},
        {"bpc", &hgm_opts::blocks_per_cu, {2, 4, 8, 16}, 0},
        {"hub", &hgm_opts::hub_threshold, {1024, 4096, 8192, 32768, 1 << 30}, 0},
        {"hot", &hgm_opts::hot_degree, {16, 64, 256}, 0},
        {"clear", &hgm_opts::clear_ratio, {2, 8, 32}, 0},
        {"first", &hgm_opts::first_batch_pct, {25, 40, 55}, 0},
        {"tail", &hgm_opts::tail_pins, {-1, 1024, 4096, 32768}, 2},
        {"bins", &hgm_opts::bin_shift, {-1, 0, 12, 13, 14}, 2},
    };
    std::vector<Knob> out;
    for (auto &x : k)
        if (x.kind == 0 || x.kind == (batch ? 1 : 2)) out.push_back(x);
    return out;
}

// Fields at the candidates that need the most workspace: the lowest hub
// threshold (the hub pieces), a solo part, a tail and bins (their size does
// not depend on the shift; the widest bins fit the most instances); every edge grid is
// sized separately (largest_size).
constexpr int32_t kMinTunedHub = 1024;

hgm_opts largest_workspace(const hgm_opts *base) {
    hgm_opts o;
    memset(&o, 0, sizeof(o));
    if (base) o = *base;
    o.hub_threshold = o.hub_threshold ? std::min(o.hub_threshold, kMinTunedHub) : kMinTunedHub;
    if (o.solo_max_kappa < 0) o.solo_max_kappa = 0;
    if (o.tail_pins <= 0) o.tail_pins = 32768;
    o.bin_shift = 14;  // bins wherever any candidate shift allows them
    return o;
}

// The library default of each field, as the value the tuner reports.
int32_t default_of(const char *name, bool batch, bool graph) {
    if (!strcmp(name, "solo")) return 0;  // by the batch's size (solo_auto_bound)
    if (!strcmp(name, "grid")) return batch ? kEdgeGridBatch : kEdgeGrid;
    if (!strcmp(name, "bpc")) return kBlocksPerCu;
    if (!strcmp(name, "hub")) return kDefaultHubThreshold;
    if (!strcmp(name, "hot")) return kHotDegree;
    if (!strcmp(name, "clear")) return kFullClearRatio;
    if (!strcmp(name, "first")) return graph ? kFirstBatchPctGraph : kFirstBatchPct;
    if (!strcmp(name, "tail")) return kDefaultTailPins;
    if (!strcmp(name, "bins")) return kDefaultBinShift;
    return 0;
}

void fill_defaults(hgm_opts *o, bool batch, bool graph) {
    for (auto &k : knobs(batch))
        if (o->*(k.field) == 0) o->*(k.field) = default_of(k.name, batch, graph);
}

// Shape bucket of a matching: device, kind, variant and layout, log2 of the
// pins, mean edge size, and for a batch log2 of the instance count.
std::string device_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    std::ostringstream s;
    s << p.gcnArchName << ":" << p.multiProcessorCount;
    std::string out = s.str();
    for (auto &c : out)
        if (c == ' ') c = '_';
    return out;
}

std::string bucket(const char *kind, const hgm_opts &o, int64_t m, int64_t kappa, int64_t count) {
    const int kb = kappa > 0 ? (int)lround(log2((double)kappa)) : 0;
    const int db = m > 0 ? (int)std::min<int64_t>(64, (kappa + m / 2) / m) : 0;
    const int cb = count > 0 ? (int)lround(log2((double)count)) : 0;
    std::ostringstream s;
    s << device_name() << " " << kind << " v" << o.variant << " p" << o.pairs << " r" << o.reseed
      << " k" << kb << " d" << db << " c" << cb;
    return s.str();
}

const char *cache_path(const char *path) {
    if (path && *path) return path;
    const char *env = getenv("HGM_TUNE_CACHE");
    return env && *env ? env : nullptr;
}

std::mutex g_cache_mu;

// The schedule fields of `o` as "name=value" words.
std::string encode(const hgm_opts &o, bool batch) {
    std::ostringstream s;
    for (auto &k : knobs(batch)) s << " " << k.name << "=" << o.*(k.field);
    return s.str();
}

// Writes or replaces the line of `key` in the cache file.
int cache_put(const char *path, const std::string &key, const hgm_opts &o, bool batch,
              double ms_default, double ms_best) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::vector<std::string> lines;
    {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line))
            if (line.compare(0, key.size() + 3, key + " : ") != 0 && !line.empty())
                lines.push_back(line);
    }
    std::ostringstream l;
    l << key << " :" << encode(o, batch) << " ms_default=" << ms_default << " ms_tuned=" << ms_best;
    lines.push_back(l.str());
    std::ofstream out(path, std::ios::trunc);
    if (!out) return HGM_E_ARG;
    for (auto &x : lines) out << x << "\n";
    return out ? HGM_OK : HGM_E_ARG;
}

// Reads the schedule of `key` into o (its other fields untouched).
int cache_get(const char *path, const std::string &key, hgm_opts *o, bool batch) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ifstream in(path);
    if (!in) return HGM_E_ARG;
    std::string line;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size() + 3, key + " : ") != 0) continue;
        std::istringstream words(line.substr(key.size() + 3));
        std::string w;
        hgm_opts t = *o;
        while (words >> w) {
            const size_t eq = w.find('=');
            if (eq == std::string::npos) continue;
            const std::string name = w.substr(0, eq);
            for (auto &k : knobs(batch))
                if (name == k.name) t.*(k.field) = (int32_t)strtol(w.c_str() + eq + 1, nullptr, 10);
        }
        *o = t;
        return HGM_OK;
    }
    return HGM_E_ARG;
}

// Coordinate descent over the knobs.  run(o) performs one matching with
// options o and returns an HGM code; snapshot(true) copies the output as the
// reference after the starting schedule's first run, snapshot(false)
// compares a candidate's output with it (1 when they differ).
int search(bool batch, bool graph, const hgm_opts *base, int reps,
           const std::function<int(const hgm_opts &)> &run,
           const std::function<int(bool)> &snapshot,  // true: keep as reference; false: compare
           hgm_opts *best, hgm_tune_report *rep) {
    if (reps < 1) reps = 1;
    hgm_opts cur;
    memset(&cur, 0, sizeof(cur));
    if (base) cur = *base;
    fill_defaults(&cur, batch, graph);
    int evaluations = 0, identical = 1;
    auto time_of = [&](const hgm_opts &o, double *ms, bool reference) -> int {
        int rc = run(o);  // untimed first call, also the bitmap check
        if (rc != HGM_OK) return rc;
        rc = snapshot(reference);
        if (rc != HGM_OK) return rc;
        std::vector<double> t;
        for (int i = 0; i < reps; ++i) {
            const double t0 = now_s();
            rc = run(o);
            if (rc != HGM_OK) return rc;
            t.push_back((now_s() - t0) * 1e3);
        }
        std::sort(t.begin(), t.end());
        *ms = t[t.size() / 2];
        evaluations += 1;
        return HGM_OK;
    };
    double best_ms = 0.0;
    int rc = time_of(cur, &best_ms, true);
    if (rc != HGM_OK) return rc;
    const double ms_default = best_ms;
    for (auto &k : knobs(batch)) {
        int32_t keep = cur.*(k.field);
        for (int32_t v : k.values) {
            if (v == keep) continue;
            hgm_opts cand = cur;
            cand.*(k.field) = v;
            double ms = 0.0;
            rc = time_of(cand, &ms, false);
            if (rc == 1) {  // bitmap differs from the reference: never chosen
                identical = 0;
                continue;
            }
            if (rc != HGM_OK) return rc;
            if (ms < best_ms * 0.98) {
                best_ms = ms;
                keep = v;
            }
        }
        cur.*(k.field) = keep;
    }
    *best = cur;
    if (rep) {
        rep->ms_default = ms_default;
        rep->ms_best = best_ms;
        rep->evaluations = evaluations;
        rep->identical = identical;
    }
    return HGM_OK;
}

// Host copy of a device bitmap for the candidate check.
struct BitsCheck {
    const uint32_t *dev;
    size_t words;
    hipStream_t stream;
    std::vector<uint32_t> ref, cur;
    int operator()(bool reference) {
        std::vector<uint32_t> &dst = reference ? ref : cur;
        dst.assign(words, 0);
        if (words && (hipMemcpyAsync(dst.data(), dev, 4 * words, hipMemcpyDeviceToHost, stream) !=
                          hipSuccess ||
                      hipStreamSynchronize(stream) != hipSuccess))
            return HGM_E_HIP;
        if (reference) return HGM_OK;
        return cur == ref ? HGM_OK : 1;
    }
};

// The largest workspace any candidate needs: the list capacity is not
// monotone in the edge grid (it rounds the edges per workgroup up to whole
// chunks), so every candidate grid is sized.
template <typename F>
size_t largest_size(const hgm_opts *base, bool batch, F size_of) {
    size_t best = size_of(base);
    if (!best) return 0;
    hgm_opts o = largest_workspace(base);
    for (auto &k : knobs(batch)) {
        if (strcmp(k.name, "grid")) continue;
        for (int32_t v : k.values) {
            o.edge_grid = v;
            const size_t x = size_of(&o);
            if (!x) return 0;
            best = std::max(best, x);
        }
    }
    return best;
}

}  // namespace

extern "C" {

size_t hgm_tune_workspace_size(const hgm_csr *g, const hgm_opts *base) {
    return largest_size(base, false, [&](const hgm_opts *o) { return hgm_workspace_size(g, o); });
}

size_t hgm_tune_batch_workspace_size(const hgm_batch *b, const hgm_opts *base) {
    return largest_size(base, true,
                        [&](const hgm_opts *o) { return hgm_batch_workspace_size(b, o); });
}

int hgm_tune(const hgm_csr *g, uint32_t seed, uint32_t *matched_bits, void *workspace,
             size_t ws_bytes, const hgm_opts *base, void *stream, int32_t reps,
             const char *cache, hgm_opts *best, hgm_tune_report *report) {
    if (!g || !best || reps < 0) return HGM_E_ARG;
    if (ws_bytes < hgm_tune_workspace_size(g, base)) return HGM_E_SIZE;
    const bool graph = base && base->pairs;
    BitsCheck check{matched_bits, (size_t)((int64_t)g->m + 31) / 32, (hipStream_t)stream, {}, {}};
    auto run = [&](const hgm_opts &o) {
        return hgm_match(g, seed, matched_bits, workspace, ws_bytes, &o, stream, nullptr);
    };
    int rc = search(false, graph, base, reps, run, std::ref(check), best, report);
    if (rc != HGM_OK) return rc;
    const char *path = cache_path(cache);
    if (path)
        rc = cache_put(path, bucket("match", *best, g->m, g->kappa, 0), *best, false,
                       report ? report->ms_default : 0.0, report ? report->ms_best : 0.0);
    return rc;
}

int hgm_tune_batch(const hgm_batch *b, uint32_t *matched_bits, void *workspace, size_t ws_bytes,
                   const hgm_opts *base, void *stream, int32_t reps, const char *cache,
                   hgm_opts *best, hgm_tune_report *report) {
    if (!b || !best || reps < 0) return HGM_E_ARG;
    if (ws_bytes < hgm_tune_batch_workspace_size(b, base)) return HGM_E_SIZE;
    BitsCheck check{matched_bits, (size_t)b->words_total, (hipStream_t)stream, {}, {}};
    auto run = [&](const hgm_opts &o) {
        return hgm_match_batch(b, matched_bits, workspace, ws_bytes, &o, stream, nullptr);
    };
    int rc = search(true, false, base, reps, run, std::ref(check), best, report);
    if (rc != HGM_OK) return rc;
    const char *path = cache_path(cache);
    if (path)
        rc = cache_put(path, bucket("batch", *best, b->m_total, b->kappa_total, b->count), *best,
                       true, report ? report->ms_default : 0.0, report ? report->ms_best : 0.0);
    return rc;
}

int hgm_tuned_opts(const char *cache, const hgm_csr *g, hgm_opts *opts) {
    if (!g || !opts) return HGM_E_ARG;
    const char *path = cache_path(cache);
    if (!path) return HGM_E_ARG;
    return cache_get(path, bucket("match", *opts, g->m, g->kappa, 0), opts, false);
}

int hgm_tuned_batch_opts(const char *cache, const hgm_batch *b, hgm_opts *opts) {
    if (!b || !opts) return HGM_E_ARG;
    const char *path = cache_path(cache);
    if (!path) return HGM_E_ARG;
    return cache_get(path, bucket("batch", *opts, b->m_total, b->kappa_total, b->count), opts,
                     true);
}

}  // extern "C"
