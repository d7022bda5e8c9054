// C interface of hgm (include/hgm.h): argument checks, workspace layout and
// the host round loop.  Every step of the matching runs in kernels.hip; this
// file only enqueues them and reads the per-round counters back.
#include <string.h>

#include <algorithm>
#include <vector>

#include "hgm.h"
#include "internal.h"

using namespace hgm;

namespace {

constexpr int kDefaultRoundsPerSync = 4;
constexpr int kMaxRoundsPerSync = 200;
constexpr int kDefaultHubThreshold = 8192;
constexpr int kBlocksPerCu = 8;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t key, best0, best1, done, list0, list1, slots, err, live_key, hubs, hub_count,
        hub_piece_off, vbits, total;
    int ring;
};

struct Opts {
    int variant, hub_threshold, rounds_per_sync, validate, max_rounds;
};

int resolve_opts(const hgm_opts *in, Opts *o) {
    hgm_opts d;
    memset(&d, 0, sizeof(d));
    if (in) d = *in;
    if (d.variant < HGM_VARIANT_AUTO || d.variant > HGM_VARIANT_CREW) return HGM_E_ARG;
    if (d.hub_threshold < 0 || d.rounds_per_sync < 0 || d.max_rounds < 0) return HGM_E_ARG;
    if (d.rounds_per_sync > kMaxRoundsPerSync) return HGM_E_ARG;
    o->variant = d.variant;
    o->hub_threshold = d.hub_threshold ? d.hub_threshold : kDefaultHubThreshold;
    o->rounds_per_sync = d.rounds_per_sync ? d.rounds_per_sync : kDefaultRoundsPerSync;
    o->validate = d.validate != 0;
    o->max_rounds = d.max_rounds;
    return HGM_OK;
}

// Whether the vertex-centric form runs in round r.
bool crew_round(const Opts &o, int r) {
    (void)r;
    return o.variant == HGM_VARIANT_CREW;
}

bool uses_crew(const Opts &o) { return o.variant == HGM_VARIANT_CREW; }

Layout make_layout(int64_t n, int64_t m, int64_t kappa, const Opts &o) {
    Layout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t p = at;
        at = align256(at + std::max<size_t>(bytes, 1));
        return p;
    };
    L.ring = o.rounds_per_sync + 2;
    L.key = take(8 * (size_t)m);
    L.best0 = take(8 * (size_t)n);
    L.best1 = take(8 * (size_t)n);
    L.done = take((size_t)n);
    L.list0 = take(4 * (size_t)m);
    L.list1 = take(4 * (size_t)m);
    L.slots = take(sizeof(RoundSlot) * (size_t)L.ring);
    L.err = take(4);
    const bool crew = uses_crew(o);
    L.live_key = take(crew ? 8 * (size_t)m : 0);
    L.hubs = take(crew ? 4 * (size_t)n : 0);
    L.hub_count = take(4);
    L.hub_piece_off = take(crew ? 4 * ((size_t)n + 1) : 0);
    L.vbits = take(o.validate ? 4 * (size_t)((kappa + 31) / 32) : 0);
    L.total = at;
    return L;
}

State carve(void *ws, const Layout &L) {
    char *b = (char *)ws;
    State s;
    s.key = (uint64_t *)(b + L.key);
    s.best[0] = (uint64_t *)(b + L.best0);
    s.best[1] = (uint64_t *)(b + L.best1);
    s.done = (uint8_t *)(b + L.done);
    s.list[0] = (int32_t *)(b + L.list0);
    s.list[1] = (int32_t *)(b + L.list1);
    s.slots = (RoundSlot *)(b + L.slots);
    s.ring = L.ring;
    s.err = (int32_t *)(b + L.err);
    s.live_key = (uint64_t *)(b + L.live_key);
    s.hubs = (int32_t *)(b + L.hubs);
    s.hub_count = (int32_t *)(b + L.hub_count);
    s.hub_piece_off = (int32_t *)(b + L.hub_piece_off);
    s.vbits = (uint32_t *)(b + L.vbits);
    return s;
}

int check_graph(const hgm_csr *g, const Opts &o) {
    if (!g) return HGM_E_ARG;
    if (g->n < 0 || g->m < 0 || g->kappa < 0) return HGM_E_ARG;
    if (g->kappa >= ((int64_t)1 << 31)) return HGM_E_SIZE;
    if (g->m > 0 && (!g->e_off || !g->w)) return HGM_E_ARG;
    if (g->kappa > 0 && !g->e_pins) return HGM_E_ARG;
    if (g->kappa > 0 && g->m == 0) return HGM_E_ARG;
    if (uses_crew(o) || o.validate) {
        if (!g->v_off) return HGM_E_ARG;
        if (g->kappa > 0 && (!g->v_edges || g->n == 0)) return HGM_E_ARG;
    }
    return HGM_OK;
}

int device_grid() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 0;
    int grid = cus * kBlocksPerCu;
    if (dev >= 0 && dev < 64) cached[dev] = grid;
    return grid;
}

#define HGM_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return HGM_E_HIP;     \
    } while (0)

}  // namespace

extern "C" {

int hgm_version(void) { return 100; }

const char *hgm_strerror(int code) {
    switch (code) {
    case HGM_OK: return "success";
    case HGM_E_ARG: return "invalid argument (NULL pointer with non-zero size, negative size or bad option)";
    case HGM_E_CSR: return "malformed hypergraph (offsets, ids, repeated pins or vertex side not the transpose)";
    case HGM_E_SIZE: return "size limit: kappa >= 2^31 or workspace too small";
    case HGM_E_ROUND_LIMIT: return "round limit reached with live edges remaining";
    case HGM_E_HIP: return "HIP runtime error";
    default: return "unknown error code";
    }
}

size_t hgm_workspace_size(const hgm_csr *g, const hgm_opts *opts) {
    Opts o;
    if (resolve_opts(opts, &o) != HGM_OK || !g) return 0;
    if (g->n < 0 || g->m < 0 || g->kappa < 0 || g->kappa >= ((int64_t)1 << 31)) return 0;
    return make_layout(g->n, g->m, g->kappa, o).total;
}

int hgm_match(const hgm_csr *gin, uint32_t seed, uint32_t *matched_bits, void *workspace,
              size_t ws_bytes, const hgm_opts *opts, void *stream, hgm_stats *stats) {
    Opts o;
    int rc = resolve_opts(opts, &o);
    if (rc != HGM_OK) return rc;
    rc = check_graph(gin, o);
    if (rc != HGM_OK) return rc;
    if (gin->m > 0 && !matched_bits) return HGM_E_ARG;
    if (stats && stats->cap > 0 &&
        (!stats->live_edges || !stats->live_pins || !stats->matched_per_round))
        return HGM_E_ARG;
    const Layout lay = make_layout(gin->n, gin->m, gin->kappa, o);
    if (!workspace) return HGM_E_ARG;
    if (ws_bytes < lay.total) return HGM_E_SIZE;
    if (((uintptr_t)workspace & 255) != 0) return HGM_E_ARG;

    Graph g;
    g.n = gin->n;
    g.m = gin->m;
    g.kappa = gin->kappa;
    g.e_off = gin->e_off;
    g.e_pins = gin->e_pins;
    g.v_off = gin->v_off;
    g.v_edges = gin->v_edges;
    g.w = gin->w;
    const State s = carve(workspace, lay);
    Launch L;
    L.grid = device_grid();
    L.stream = (hipStream_t)stream;
    if (L.grid <= 0) return HGM_E_HIP;

    const bool crew = uses_crew(o);
    HGM_TRY(launch_init(L, g, seed, s, matched_bits, crew ? 1 : 0));
    if (o.validate) {
        HGM_TRY(launch_validate(L, g, s, 1));
        int32_t err = 0;
        HGM_TRY(hipMemcpyAsync(&err, s.err, sizeof(err), hipMemcpyDeviceToHost, L.stream));
        HGM_TRY(hipStreamSynchronize(L.stream));
        if (err) return HGM_E_CSR;
    }

    std::vector<RoundSlot> ring(lay.ring);
    std::vector<int64_t> live_e, live_p, matched_r;
    std::vector<uint64_t> weight_r;
    live_e.push_back(g.m);
    live_p.push_back(g.kappa);

    int rounds = 0;
    bool finished = g.m == 0;
    if (!finished) {
        if (crew_round(o, 0))
            HGM_TRY(launch_vertex_max(L, g, s, 0, o.hub_threshold));
        else
            HGM_TRY(launch_scatter(L, g, s, 0));
    }
    int launched = 0;  // rounds whose test has been enqueued
    while (!finished) {
        int batch = o.rounds_per_sync;
        if (o.max_rounds > 0) batch = std::min(batch, o.max_rounds - launched);
        if (batch <= 0) return HGM_E_ROUND_LIMIT;
        const int first = launched;
        for (int b = 0; b < batch; ++b) {
            const int r = launched;
            const bool next_crew = crew_round(o, r + 1);
            const bool cur_crew = crew_round(o, r);
            // Clear the next round's max buffer when the next round scatters
            // (always in CRCW; at the switch from CREW to CRCW).
            HGM_TRY(launch_test(L, g, s, r, next_crew ? 0 : 1, matched_bits));
            (void)cur_crew;
            HGM_TRY(launch_retire(L, g, s, r + 1, next_crew ? 0 : 1));
            if (next_crew) HGM_TRY(launch_vertex_max(L, g, s, r + 1, o.hub_threshold));
            launched += 1;
        }
        HGM_TRY(hipMemcpyAsync(ring.data(), s.slots, sizeof(RoundSlot) * lay.ring,
                               hipMemcpyDeviceToHost, L.stream));
        HGM_TRY(hipStreamSynchronize(L.stream));
        for (int r = first; r < launched; ++r) {
            const RoundSlot &cur = ring[r % lay.ring];
            const RoundSlot &nxt = ring[(r + 1) % lay.ring];
            matched_r.push_back(cur.matched);
            weight_r.push_back(cur.weight);
            if (nxt.live == 0) {
                finished = true;
                rounds = r + 1;
                break;
            }
            live_e.push_back(nxt.live);
            live_p.push_back(nxt.kappa);
        }
        if (!finished && o.max_rounds > 0 && launched >= o.max_rounds) return HGM_E_ROUND_LIMIT;
    }

    if (stats) {
        stats->rounds = rounds;
        int64_t tm = 0;
        uint64_t tw = 0;
        for (int r = 0; r < rounds; ++r) {
            tm += matched_r[r];
            tw += weight_r[r];
            if (r < stats->cap) {
                stats->live_edges[r] = live_e[r];
                stats->live_pins[r] = live_p[r];
                stats->matched_per_round[r] = matched_r[r];
            }
        }
        stats->matched = tm;
        stats->weight = tw;
    }
    return HGM_OK;
}

}  // extern "C"
