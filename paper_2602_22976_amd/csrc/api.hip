// C interface of hgm (include/hgm.h): argument checks, workspace layout and
// the host round loop.  Every step of the matching runs in kernels.hip; this
// file only enqueues them and reads the per-round counters back.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>

#include "hgm.h"
#include "internal.h"
#include "schedule.h"

using namespace hgm;

namespace {

constexpr int kFirstBatch = 4;         // fewest rounds enqueued before the first termination check
constexpr int kAdaptiveMaxBatch = 32;  // cap of a predicted batch
constexpr int kMaxRoundsPerSync = 200;
// Per-round shrink of the live pins assumed before two counts are known (the
// measured ratio on the synthetic workloads lies between 0.2 and 0.35 in the
// early rounds).
constexpr double kPriorShrink = 0.3;
// Rounds of per-round sums the solo part records (later rounds of a solo
// instance count in the totals only).
constexpr int kSoloRounds = 1 << 16;
// The tail takes at most this many live edges.
constexpr int kTailCap = 1 << 16;
// Rows of the tail record copied with the round counters at each check.
constexpr int kTailRowsFirst = 64;
// Binned maximum: a round uses it when the host expects at least n / 2
// surviving pins (below that the reduction's fixed cost, one launch and a
// pass over every bin, outweighs the atomics it saves).  bin_shift 0
// (automatic): instances of at least these sizes, bins of 2^(ceil(log2 n) -
// 7) vertices (about 128 bins) clamped to [2^12, 2^14], and on the device
// only where the degree profile sent round 0 to the vertex form.
constexpr int64_t kBinAutoMinN = (int64_t)1 << 17;
constexpr int64_t kBinAutoMinKappa = (int64_t)1 << 20;
constexpr int kBinAutoLo = 12, kBinAutoHi = 14;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    bool stored_keys;  // batch: keys precomputed per instance
    size_t key, eseed, best0, best1, done, list0, list1, cnt0, cnt1, rec[2][5], stats, err, live_key, vedges0,
        vedges1, vlen0, vlen1, pieces,
        piece_count, hot, wrange, vbits, goff, vbase, bitoff, gvoff, ebase, solo, tail_list[2][4],
        tail, bin_v, bin_key, bin_cursor, total;
    int ring, grid, region, piece_cap, solo_rounds, tail_cap, bin_rb, bin_nb;
};

// Edge schedule: `grid` workgroups, each owning `region` consecutive edge ids
// (a multiple of kBlock); grid * region >= m.
void edge_schedule(int64_t m, int edge_grid, int *grid, int *region) {
    const int64_t chunks = std::max<int64_t>(1, (m + kBlock - 1) / kBlock);
    const int64_t g = std::min<int64_t>(edge_grid, chunks);
    *grid = (int)g;
    *region = (int)(((chunks + g - 1) / g) * kBlock);
}

struct Opts {
    int variant, hub_threshold, rounds_per_sync, validate, max_rounds;
    int64_t solo_max_kappa;  // batches: solo part bound (-1: no solo part, 0: by size)
    int edge_grid, blocks_per_cu, clear_ratio, hot_degree, first_batch_pct;  // 0 = per kind
    int64_t tail_pins;  // one instance: tail bound (-1: no tail)
    int bin_shift;      // binned maximum: log2 vertices per bin, 0 automatic, -1 off
    bool reseed;            // priorities redrawn every round (round_seed)
    bool pairs;             // graph: two pins per edge at e_pins[2e], no offsets
    bool adaptive;          // rounds_per_sync chosen per batch from the decay of live pins
    bool have_vertex_side;  // v_off / v_edges given
};

int resolve_opts(const hgm_opts *in, Opts *o) {
    hgm_opts d;
    memset(&d, 0, sizeof(d));
    if (in) d = *in;
    if (d.variant < HGM_VARIANT_AUTO || d.variant > HGM_VARIANT_CREW) return HGM_E_ARG;
    if (d.hub_threshold < 0 || d.rounds_per_sync < 0 || d.max_rounds < 0) return HGM_E_ARG;
    if (d.rounds_per_sync > kMaxRoundsPerSync) return HGM_E_ARG;
    if (d.reseed != 0 && d.reseed != 1) return HGM_E_ARG;
    if (d.pairs != 0 && d.pairs != 1) return HGM_E_ARG;
    // The pair layout has no edge offsets for the CREW rounds' edge-side passes
    // to share; graphs run the edge-centric rounds.
    if (d.pairs && d.variant == HGM_VARIANT_CREW) return HGM_E_ARG;
    o->variant = d.variant;
    o->hub_threshold = d.hub_threshold ? d.hub_threshold : kDefaultHubThreshold;
    o->adaptive = d.rounds_per_sync == 0;
    o->rounds_per_sync = d.rounds_per_sync ? d.rounds_per_sync : kAdaptiveMaxBatch;
    o->validate = d.validate != 0;
    o->max_rounds = d.max_rounds;
    o->reseed = d.reseed != 0;
    o->pairs = d.pairs != 0;
    if (d.solo_max_kappa < -1) return HGM_E_ARG;
    o->solo_max_kappa = d.solo_max_kappa;  // 0: solo_auto_bound of the batch's pins
    if (d.edge_grid < 0 || d.edge_grid > 65536 || d.blocks_per_cu < 0 || d.blocks_per_cu > 32 ||
        d.clear_ratio < 0 || d.clear_ratio > (1 << 20) || d.hot_degree < 0 ||
        d.first_batch_pct < 0 || d.first_batch_pct > 400)
        return HGM_E_ARG;
    o->edge_grid = d.edge_grid;  // 0: per kind (make_layout)
    o->blocks_per_cu = d.blocks_per_cu ? d.blocks_per_cu : kBlocksPerCu;
    o->clear_ratio = d.clear_ratio ? d.clear_ratio : kFullClearRatio;
    o->hot_degree = d.hot_degree ? d.hot_degree : kHotDegree;
    o->first_batch_pct = d.first_batch_pct;  // 0: resolved per instance (graphs differ)
    if (d.tail_pins < -1) return HGM_E_ARG;
    o->tail_pins = d.tail_pins == 0 ? kDefaultTailPins : d.tail_pins;
    if (d.bin_shift != -1 && d.bin_shift != 0 &&
        (d.bin_shift < kBinMinShift || d.bin_shift > kBinMaxShift))
        return HGM_E_ARG;
    o->bin_shift = d.bin_shift;
    return HGM_OK;
}

// Whether the vertex-centric form runs in round r.  AUTO: round 0, where every
// edge is live and the vertex pass needs no atomics, when the vertex side is
// given; the edge-centric form afterwards, since it touches only the pins of
// live edges while the vertex pass would scan every open vertex's full list.
bool crew_round(const Opts &o, int r) {
    if (o.variant == HGM_VARIANT_CREW) return true;
    if (o.variant == HGM_VARIANT_AUTO) return r == 0 && o.have_vertex_side;
    return false;
}

bool any_crew_round(const Opts &o) { return crew_round(o, 0); }
bool uses_live_key(const Opts &o) { return o.variant == HGM_VARIANT_CREW; }

// log2 of the vertices per bin of the binned maximum, or 0 without bins.  It
// needs the vertex side (the bins' capacities are degree sums, v_off), hub
// pieces (hub pins stay out of the bins) and the CRCW rounds' offset layout
// of one instance: AUTO with the vertex side.
int bin_shift_for(int64_t n, int64_t kappa, const Opts &o, bool batch) {
    if (batch || o.pairs || o.variant != HGM_VARIANT_AUTO || !o.have_vertex_side ||
        o.bin_shift < 0 || n <= 0 || kappa <= 0)
        return 0;
    int rb = o.bin_shift;
    if (rb == 0) {  // automatic: large instances, about 128 bins
        if (n < kBinAutoMinN || kappa < kBinAutoMinKappa) return 0;
        int lg = 0;
        while (((int64_t)1 << lg) < n) ++lg;
        rb = std::min(kBinAutoHi, std::max(kBinAutoLo, lg - 7));
    }
    const int64_t nb = (n + ((int64_t)1 << rb) - 1) >> rb;
    return nb <= kBinMaxBins ? rb : 0;
}

Layout make_layout(int64_t n, int64_t m, int64_t kappa, const Opts &o, bool batch = false) {
    Layout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t p = at;
        at = align256(at + std::max<size_t>(bytes, 1));
        return p;
    };
    L.ring = o.rounds_per_sync + 2;
    edge_schedule(m, o.edge_grid ? o.edge_grid : batch ? kEdgeGridBatch : kEdgeGrid, &L.grid,
                  &L.region);
    const size_t cap = (size_t)L.grid * (size_t)L.region;
    L.stored_keys = batch;
    L.key = take(batch ? 8 * (size_t)m : 0);
    L.eseed = take(batch && o.reseed ? 8 * (size_t)m : 0);
    L.best0 = take(8 * (size_t)n);
    L.best1 = take(8 * (size_t)n);
    L.done = take((size_t)n);
    L.list0 = take(4 * cap);
    L.list1 = take(4 * cap);
    L.cnt0 = take(4 * (size_t)L.grid);
    L.cnt1 = take(4 * (size_t)L.grid);
    for (int k = 0; k < 2; ++k) {
        L.rec[k][0] = take(4 * cap);                 // rec_a
        L.rec[k][1] = take(4 * cap);                 // rec_b
        L.rec[k][2] = take(4 * cap);                 // rec_c
        L.rec[k][3] = take(batch ? 4 * cap : 0);     // rec_vb
        L.rec[k][4] = take(8 * cap);                 // rec_key
    }
    L.stats = take(sizeof(RoundStats) * (size_t)L.ring);
    L.err = take(4);
    L.live_key = take(uses_live_key(o) ? 8 * (size_t)m : 0);
    // CREW: incidence lists compacted every round, double-buffered.
    L.vedges0 = take(uses_live_key(o) ? 4 * (size_t)kappa : 0);
    L.vedges1 = take(uses_live_key(o) ? 4 * (size_t)kappa : 0);
    L.vlen0 = take(uses_live_key(o) ? 4 * (size_t)n : 0);
    L.vlen1 = take(uses_live_key(o) ? 4 * (size_t)n : 0);
    // pieces: each vertex of degree d > T gives ceil(d / P) <= d / P + 1 pieces,
    // and there are fewer than kappa / T such vertices.
    L.piece_cap = any_crew_round(o)
                      ? (int)std::min<int64_t>(kappa / kHubPiece + kappa / o.hub_threshold + 1,
                                               ((int64_t)1 << 31) - 1)
                      : 0;
    L.pieces = take(sizeof(int2) * (size_t)L.piece_cap);
    L.piece_count = take(4);
    L.hot = take(8 * (size_t)kSub);
    L.wrange = take(8 * (size_t)kSub);
    L.vbits = take(o.validate ? 4 * (size_t)((kappa + 31) / 32) : 0);
    // Batch: global offsets and per-edge / per-vertex bases (see Graph).
    L.goff = take(batch ? 4 * ((size_t)m + 1) : 0);
    L.vbase = take(batch ? 4 * (size_t)m : 0);
    L.bitoff = take(batch ? 4 * (size_t)m : 0);
    L.gvoff = take(batch && o.have_vertex_side ? 4 * ((size_t)n + 1) : 0);
    L.ebase = take(batch && o.have_vertex_side ? 4 * (size_t)n : 0);
    // An instance needs at most as many rounds as it has edges (each round
    // matches its largest live edge).
    L.solo_rounds = batch && o.solo_max_kappa >= 0
                        ? (int)std::min<int64_t>(kSoloRounds, std::max<int64_t>(m, 1))
                        : 0;
    L.solo = take(L.solo_rounds ? 8 * ((size_t)kSoloHeader + 5 * (size_t)L.solo_rounds) : 0);
    // One instance: the tail's compact lists (id, pin offset or first pin,
    // count or second pin, key; two buffers) and its record.
    L.tail_cap = !batch && o.tail_pins > 0 ? (int)std::min<int64_t>(kTailCap, std::max<int64_t>(m, 1))
                                           : 0;
    for (int k = 0; k < 2; ++k)
        for (int f = 0; f < 4; ++f)
            L.tail_list[k][f] = take((f == 3 ? 8 : 4) * (size_t)L.tail_cap);
    L.tail = take(L.tail_cap ? 8 * ((size_t)kTailHeader + 5 * ((size_t)L.tail_cap + 2)) : 0);
    // Binned maximum: records (index in bin, key) at the bins' degree-sum
    // offsets, and a cursor per bin.
    L.bin_rb = bin_shift_for(n, kappa, o, batch);
    L.bin_nb = L.bin_rb ? (int)((n + ((int64_t)1 << L.bin_rb) - 1) >> L.bin_rb) : 0;
    L.bin_v = take(L.bin_nb ? 2 * (size_t)kappa : 0);
    L.bin_key = take(L.bin_nb ? 8 * (size_t)kappa : 0);
    L.bin_cursor = take(L.bin_nb ? 4 * (size_t)kBinMaxBins : 0);  // same size for every shift
    L.total = at;
    return L;
}

State carve(void *ws, const Layout &L, const Opts &o) {
    char *b = (char *)ws;
    State s;
    s.key = L.stored_keys ? (uint64_t *)(b + L.key) : nullptr;
    s.eseed = L.stored_keys && o.reseed ? (uint64_t *)(b + L.eseed) : nullptr;
    s.best[0] = (uint64_t *)(b + L.best0);
    s.best[1] = (uint64_t *)(b + L.best1);
    s.done = (uint8_t *)(b + L.done);
    s.list[0] = (int32_t *)(b + L.list0);
    s.list[1] = (int32_t *)(b + L.list1);
    s.cnt[0] = (int32_t *)(b + L.cnt0);
    s.cnt[1] = (int32_t *)(b + L.cnt1);
    for (int k = 0; k < 2; ++k) {
        s.rec_a[k] = (int32_t *)(b + L.rec[k][0]);
        s.rec_b[k] = (int32_t *)(b + L.rec[k][1]);
        s.rec_c[k] = (int32_t *)(b + L.rec[k][2]);
        s.rec_vb[k] = (int32_t *)(b + L.rec[k][3]);
        s.rec_key[k] = (uint64_t *)(b + L.rec[k][4]);
    }
    s.stats = (RoundStats *)(b + L.stats);
    s.ring = L.ring;
    s.grid = L.grid;
    s.region = L.region;
    s.err = (int32_t *)(b + L.err);
    s.live_key = (uint64_t *)(b + L.live_key);
    const bool lists = uses_live_key(o);
    s.vedges[0] = lists ? (int32_t *)(b + L.vedges0) : nullptr;
    s.vedges[1] = lists ? (int32_t *)(b + L.vedges1) : nullptr;
    s.vlen[0] = lists ? (int32_t *)(b + L.vlen0) : nullptr;
    s.vlen[1] = lists ? (int32_t *)(b + L.vlen1) : nullptr;
    s.pieces = (int2 *)(b + L.pieces);
    s.piece_count = (int32_t *)(b + L.piece_count);
    s.hot = (unsigned long long *)(b + L.hot);
    s.wrange = (uint32_t *)(b + L.wrange);
    s.piece_cap = L.piece_cap;
    s.hub_threshold = o.hub_threshold;
    s.hot_degree = o.hot_degree;
    s.vbits = (uint32_t *)(b + L.vbits);
    s.explicit0 = L.solo_rounds > 0;
    s.solo = L.solo_rounds ? (unsigned long long *)(b + L.solo) : nullptr;
    s.solo_rounds = L.solo_rounds;
    for (int k = 0; k < 2; ++k) {
        s.tail_e[k] = (int32_t *)(b + L.tail_list[k][0]);
        s.tail_a[k] = (int32_t *)(b + L.tail_list[k][1]);
        s.tail_b[k] = (int32_t *)(b + L.tail_list[k][2]);
        s.tail_key[k] = (uint64_t *)(b + L.tail_list[k][3]);
    }
    s.tail = L.tail_cap ? (unsigned long long *)(b + L.tail) : nullptr;
    s.tail_cap = L.tail_cap;
    s.tail_pins = o.tail_pins;
    s.bin_v = L.bin_nb ? (uint16_t *)(b + L.bin_v) : nullptr;
    s.bin_key = L.bin_nb ? (uint64_t *)(b + L.bin_key) : nullptr;
    s.bin_cursor = L.bin_nb ? (uint32_t *)(b + L.bin_cursor) : nullptr;
    s.bin_rb = L.bin_rb;
    s.bin_nb = L.bin_nb;
    s.bin_auto = o.bin_shift == 0;
    return s;
}

// Rounds to enqueue before the next termination check.  The first batch is
// sized from kappa: about 0.4 log2(kappa) rounds covered the measured round
// counts of hash-ordered hypergraphs (6 at kappa = 1.4e5 to 11 at 4.8e8)
// within two; graphs (every edge two pins) finish sooner, and 0.35 log2(kappa)
// matched Delaunay and random geometric graphs of 2^20 vertices (7 and 8
// rounds) within one.  Afterwards live pins shrink by a factor per round that grows
// as the instance thins out, so with the latest factor f the rounds left are
// at most about log(kappa_r) / log(f); a little over half of that, plus the
// retire pass that finds the live set empty, matched the measured counts.
// An unneeded round costs two near-empty launches (about 10 us), a missing
// one a further host round trip (about 45 us).
int next_batch(const Opts &o, int launched, const std::vector<int64_t> &live_pins, bool graph) {
    if (!o.adaptive) return o.rounds_per_sync;
    if (launched == 0 || live_pins.size() < 2) {
        const double k0 = live_pins.empty() ? 2.0 : std::max<double>(2.0, (double)live_pins[0]);
        const int pct = o.first_batch_pct ? o.first_batch_pct
                        : graph            ? kFirstBatchPctGraph
                                           : kFirstBatchPct;
        const int first = (int)std::lround(pct / 100.0 * std::log2(k0));
        return std::max(kFirstBatch, std::min(kAdaptiveMaxBatch, first));
    }
    const double cur = (double)live_pins.back();
    const double prev = (double)live_pins[live_pins.size() - 2];
    if (cur <= 1.0) return 2;
    double ratio = prev > cur ? prev / cur : 1.0;
    if (ratio < 1.5) ratio = 1.5;
    const int left = (int)std::ceil(0.55 * std::log(cur) / std::log(ratio)) + 1;
    return std::max(2, std::min(kAdaptiveMaxBatch, left));
}

void bind_graph(Opts *o, const hgm_csr *g) {
    o->have_vertex_side = g && g->v_off && (g->kappa == 0 || (g->v_edges && g->n > 0));
}

int check_batch(const hgm_batch *b, const Opts &o) {
    if (!b) return HGM_E_ARG;
    if (b->count < 0 || b->n_total < 0 || b->m_total < 0 || b->kappa_total < 0 ||
        b->words_total < 0)
        return HGM_E_ARG;
    const int64_t lim = ((int64_t)1 << 31) - 1;
    if (b->n_total > lim || b->m_total > lim || b->kappa_total > lim ||
        32 * b->words_total > lim)
        return HGM_E_SIZE;
    if (b->count > 0 && (!b->v_base || !b->e_base || !b->pin_base || !b->word_base || !b->seeds))
        return HGM_E_ARG;
    if (b->m_total > 0 && (!b->e_off || !b->w)) return HGM_E_ARG;
    if (b->kappa_total > 0 && (!b->e_pins || b->m_total == 0)) return HGM_E_ARG;
    if (b->m_total > 0 && b->count == 0) return HGM_E_ARG;
    if (o.variant == HGM_VARIANT_CREW) {
        if (!b->v_off) return HGM_E_ARG;
        if (b->kappa_total > 0 && (!b->v_edges || b->n_total == 0)) return HGM_E_ARG;
    }
    if (o.validate) return HGM_E_ARG;  // validate each instance with hgm_match instead
    if (o.pairs) return HGM_E_ARG;     // batches use the offset layout
    return HGM_OK;
}

void bind_batch(Opts *o, const hgm_batch *b) {
    o->have_vertex_side =
        b && b->v_off && (b->kappa_total == 0 || (b->v_edges && b->n_total > 0));
}

int check_graph(const hgm_csr *g, const Opts &o) {
    if (!g) return HGM_E_ARG;
    if (g->n < 0 || g->m < 0 || g->kappa < 0) return HGM_E_ARG;
    if (g->kappa >= ((int64_t)1 << 31)) return HGM_E_SIZE;
    if (g->m > 0 && ((!o.pairs && !g->e_off) || !g->w)) return HGM_E_ARG;
    if (o.pairs) {
        if (g->kappa != 2 * (int64_t)g->m) return HGM_E_ARG;
        if (((uintptr_t)g->e_pins & 7) != 0) return HGM_E_ARG;  // read as int2
    }
    if (g->kappa > 0 && !g->e_pins) return HGM_E_ARG;
    if (g->kappa > 0 && g->m == 0) return HGM_E_ARG;
    if (o.variant == HGM_VARIANT_CREW || o.validate) {
        if (!g->v_off) return HGM_E_ARG;
        if (g->kappa > 0 && (!g->v_edges || g->n == 0)) return HGM_E_ARG;
    }
    return HGM_OK;
}

// Compute units of the current device (0 on a HIP error).
int device_cus() {
    static std::atomic<int> cached[64];  // zero-initialised (static storage)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 0;
    if (dev >= 0 && dev < 64) cached[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

// Workgroups of the solo kernel: one per compute unit (each holds up to the
// whole LDS of its unit).
int solo_workgroups() { return std::max(1, device_cus()); }

// Dynamic LDS of a solo workgroup on the current device: all a workgroup may
// hold less the solo kernel's own shared variables (a multiple of 256).
int solo_lds_bytes() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c) return c;
    }
    int bytes = 0;
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        bytes <= kSoloStaticLds + 16384)
        return 0;
    const int dyn = (bytes - kSoloStaticLds) & ~255;
    if (dev >= 0 && dev < 64) cached[dev].store(dyn, std::memory_order_relaxed);
    return dyn;
}

// Best-tile vertices of an instance with nv vertices (k_solo's layout: the
// done bitmask rounded up to 256 bytes, then the tile).
int solo_tile(int lds_bytes, int64_t nv) {
    const int64_t dbytes = ((4 * ((nv + 31) / 32) + 255) / 256) * 256;
    return (int)std::max<int64_t>(0, (lds_bytes - dbytes) / 8);
}

// Largest vertex count whose instance needs at most `tiles` tiles.
int solo_verts_for(int lds_bytes, int tiles) {
    int64_t lo = 0, hi = (int64_t)lds_bytes * 8;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        const int t = solo_tile(lds_bytes, mid);
        if (t > 0 && (mid + t - 1) / t <= tiles)
            lo = mid;
        else
            hi = mid - 1;
    }
    return (int)lo;
}

// Optional per-kernel timing: an event is recorded after every kernel (and
// one before the first); consecutive events bracket one kernel on the stream.
// Events are kept in a per-thread pool and reused across calls.
struct KernelTimer {
    bool on = false;
    hipStream_t stream = nullptr;
    std::vector<int> cls, round;  // per bracketed kernel
    size_t used = 0;              // events recorded since the last harvest
    static std::vector<hipEvent_t> &pool() {
        static thread_local std::vector<hipEvent_t> p;
        return p;
    }
    hipError_t event(size_t i, hipEvent_t *ev) {
        auto &p = pool();
        while (p.size() <= i) {
            hipEvent_t e;
            hipError_t rc = hipEventCreate(&e);
            if (rc != hipSuccess) return rc;
            p.push_back(e);
        }
        *ev = p[i];
        return hipSuccess;
    }
    hipError_t start() {
        if (!on) return hipSuccess;
        used = 0;
        cls.clear();
        round.clear();
        hipEvent_t e;
        hipError_t rc = event(used, &e);
        if (rc != hipSuccess) return rc;
        used = 1;
        return hipEventRecord(e, stream);
    }
    hipError_t after(int c, int r) {
        if (!on) return hipSuccess;
        hipEvent_t e;
        hipError_t rc = event(used, &e);
        if (rc != hipSuccess) return rc;
        cls.push_back(c);
        round.push_back(r);
        used += 1;
        return hipEventRecord(e, stream);
    }
    // After a stream synchronisation: add the bracketed durations of kernels
    // of rounds < live_rounds (round -1 = setup).  The next bracket starts
    // at resume(), so the host's time between batches is not charged to the
    // next batch's first kernel.
    hipError_t harvest(int live_rounds, hgm_stats *st, std::vector<float> &round_ms) {
        if (!on) return hipSuccess;
        auto &p = pool();
        for (size_t i = 0; i < cls.size(); ++i) {
            float ms = 0.f;
            hipError_t rc = hipEventElapsedTime(&ms, p[i], p[i + 1]);
            if (rc != hipSuccess) return rc;
            const int r = round[i];
            if (r >= live_rounds) continue;
            st->kernel_ms[cls[i]] += ms;
            st->kernel_launches[cls[i]] += 1;
            if (r >= 0) {
                if ((size_t)r >= round_ms.size()) round_ms.resize(r + 1, 0.f);
                round_ms[r] += ms;
            }
        }
        used = 0;
        cls.clear();
        round.clear();
        return hipSuccess;
    }
    // Records a start event when the previous ones were harvested.
    hipError_t resume() {
        if (!on || used > 0) return hipSuccess;
        hipEvent_t e;
        hipError_t rc = event(0, &e);
        if (rc != hipSuccess) return rc;
        used = 1;
        return hipEventRecord(e, stream);
    }
};

#define HGM_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return HGM_E_HIP;     \
    } while (0)

// Enqueues setup and rounds, checking termination on the host every batch of
// rounds; shared by the single-instance and the batched entry point.
int solo_workgroups();

// Rows of the solo part's per-round sums copied with its header at the first
// termination check (more only when a solo instance ran more rounds).
constexpr int kSoloRowsFirst = 64;

int run_rounds(const Graph &g, const Opts &o, const Layout &lay, const State &s, const Launch &L,
               uint32_t seed, uint32_t *matched_bits, hgm_stats *stats, const BatchIn *batch,
               const SoloArgs *solo = nullptr) {
    int init_flags = 0;
    if (uses_live_key(o)) init_flags |= kInitLiveKey | (o.reseed ? kInitLiveMark : 0);
    // Priority seed of round r.
    auto kseed = [&](int r) { return o.reseed ? round_seed(seed, r) : seed; };
    if (any_crew_round(o)) init_flags |= kInitHubs;
    // Round 0's vertex pass of one instance skips the weight gathers when all
    // weights are equal (cardinality matching); batches gather stored keys.
    // CREW: setup finds the weight range.  AUTO: the round-0 edge kernel does,
    // only when it leaves the round to the vertex form.
    if (o.variant == HGM_VARIANT_CREW && !batch) init_flags |= kInitWeightRange;
    KernelTimer T;
    T.on = stats && stats->timing;
    T.stream = L.stream;
    if (stats) {
        for (int c = 0; c < HGM_K_CLASSES; ++c) {
            stats->kernel_ms[c] = 0.0;
            stats->kernel_launches[c] = 0;
        }
    }
    std::vector<float> round_ms;
    constexpr int kSetup = -1;
    HGM_TRY(T.start());
    if (batch) HGM_TRY(launch_batch_setup(L, g, *batch, s));
    HGM_TRY(launch_init(L, g, seed, s, matched_bits, init_flags));
    HGM_TRY(T.after(HGM_K_SETUP, kSetup));
    // Solo part of a batch: small instances run every round in one workgroup
    // each; the round kernels then start from an explicit list of the rest.
    const bool explicit0 = s.explicit0 != 0;
    std::vector<unsigned long long> solo_head(kSoloHeader + 5 * (size_t)kSoloRowsFirst, 0);
    if (explicit0) {
        HGM_TRY(launch_solo(L, g, s, *solo, matched_bits, o.reseed ? 1 : 0, solo_workgroups()));
        HGM_TRY(T.after(HGM_K_SOLO, kSetup));
        HGM_TRY(launch_live0(L, g, s, *solo));
        HGM_TRY(T.after(HGM_K_SETUP, kSetup));
    }
    if (o.validate) {
        HGM_TRY(launch_validate(L, g, s, 1));
        HGM_TRY(T.after(HGM_K_SETUP, kSetup));
        int32_t err = 0;
        HGM_TRY(hipMemcpyAsync(&err, s.err, sizeof(err), hipMemcpyDeviceToHost, L.stream));
        HGM_TRY(hipStreamSynchronize(L.stream));
        HGM_TRY(T.harvest(1, stats, round_ms));
        if (err) return HGM_E_CSR;
    }

    std::vector<RoundStats> ring(lay.ring);
    std::vector<int64_t> live_e, live_p, matched_r, matched_p;
    std::vector<uint64_t> weight_r;
    live_e.push_back(g.m);
    live_p.push_back(g.kappa);

    int rounds = 0;
    int max0_event = -1;  // timer entry of the AUTO round-0 maximum (class fixed after the sync)
    bool finished = g.m == 0;
    if (!finished) {
        HGM_TRY(T.resume());
        if (o.variant == HGM_VARIANT_AUTO && o.have_vertex_side) {
            HGM_TRY(launch_max0(L, g, s, kseed(0)));
            max0_event = (int)T.cls.size();
            HGM_TRY(T.after(HGM_K_VERTEX_MAX, 0));
        } else if (crew_round(o, 0)) {
            HGM_TRY(launch_vertex_max(L, g, s, 0, kseed(0), 0));
            HGM_TRY(T.after(HGM_K_VERTEX_MAX, 0));
        } else {
            HGM_TRY(launch_scatter(L, g, s, kseed(0)));
            HGM_TRY(T.after(HGM_K_SCATTER, 0));
        }
    }
    // Live pins of round r: the count itself once the host has read it, else
    // the latest count shrunk by the latest per-round ratio (kPriorShrink
    // while only kappa is known).  It only picks the test's way of clearing,
    // which is correct either way.
    auto predicted_pins = [&](int r) -> double {
        const int known = (int)live_p.size();  // live_p[i] = kappa_i for i < known
        if (r < known) return (double)live_p[r];
        const double last = (double)live_p.back();
        if (known < 2) return last * std::pow(kPriorShrink, (double)(r - (known - 1)));
        const double prev = (double)live_p[known - 2];
        const double f = (prev > 0 && last < prev) ? last / prev : 1.0;
        return last * std::pow(f, (double)(r - (known - 1)));
    };
    int launched = 0;  // rounds whose test has been enqueued
    // The tail workgroup (one instance): launched after the retire pass of a
    // round the host expects to have at most tail_pins live pins, which then
    // ends the batch of rounds; once a launch found more, later ones do not.
    const bool tail_on = s.tail != nullptr;
    bool tail_missed = false;
    std::vector<unsigned long long> tail_head(kTailHeader + 5 * (size_t)kTailRowsFirst, 0);
    while (!finished) {
        int batch = next_batch(o, launched, live_p, g.kappa == 2 * (int64_t)g.m);
        if (o.max_rounds > 0) batch = std::min(batch, o.max_rounds - launched);
        if (batch <= 0) return HGM_E_ROUND_LIMIT;
        const int first = launched;
        bool tail_launched = false;
        HGM_TRY(T.resume());
        for (int b = 0; b < batch; ++b) {
            const int r = launched;
            const bool next_crew = crew_round(o, r + 1);
            // Clear the next round's max buffer when the next round scatters
            // (always in CRCW; at the switch from CREW to CRCW).
            const int clear = next_crew ? kClearNone
                              : predicted_pins(r) * o.clear_ratio >= (double)g.n ? kClearAll
                                                                                    : kClearPins;
            HGM_TRY(launch_test(L, g, s, r, clear, matched_bits, kseed(r)));
            HGM_TRY(T.after(HGM_K_TEST, r));
            // The next maximum by bins when the host expects at least n / 2
            // surviving pins (correct either way).
            const bool binned =
                s.bin_nb > 0 && !next_crew && 2.0 * predicted_pins(r + 1) >= (double)g.n;
            HGM_TRY(launch_retire(L, g, s, r + 1, next_crew ? 0 : 1, kseed(r + 1), o.reseed ? 1 : 0,
                                  binned ? 1 : 0));
            HGM_TRY(T.after(HGM_K_RETIRE, r));
            if (next_crew) {
                HGM_TRY(launch_vertex_max(L, g, s, r + 1, kseed(r + 1), o.reseed ? 1 : 0));
                HGM_TRY(T.after(HGM_K_VERTEX_MAX, r + 1));
            }
            launched += 1;
            if (tail_on && predicted_pins(r + 1) <= (double)o.tail_pins) {
                HGM_TRY(launch_tail(L, g, s, r + 1, matched_bits, seed, o.reseed ? 1 : 0,
                                    o.max_rounds));
                HGM_TRY(T.after(HGM_K_TAIL, r + 1));
                tail_launched = true;
                if (!tail_missed) break;
            }
        }
        // Copy the slots of rounds first .. launched (at most two ranges of the ring).
        for (int r = first; r <= launched;) {
            const int slot = r % lay.ring;
            const int run = std::min(launched - r + 1, lay.ring - slot);
            HGM_TRY(hipMemcpyAsync(&ring[slot], &s.stats[slot], sizeof(RoundStats) * run,
                                   hipMemcpyDeviceToHost, L.stream));
            r += run;
        }
        if (explicit0 && first == 0)
            HGM_TRY(hipMemcpyAsync(solo_head.data(), s.solo,
                                   sizeof(unsigned long long) * solo_head.size(),
                                   hipMemcpyDeviceToHost, L.stream));
        if (tail_launched)
            HGM_TRY(hipMemcpyAsync(tail_head.data(), s.tail,
                                   sizeof(unsigned long long) * tail_head.size(),
                                   hipMemcpyDeviceToHost, L.stream));
        HGM_TRY(hipStreamSynchronize(L.stream));
        // A bin that overflowed means v_off does not describe e_pins' transpose.
        for (int r = first; r <= launched; ++r)
            if (ring[r % lay.ring].bin_overflow) return HGM_E_CSR;
        auto sum = [](const unsigned long long *a) {
            unsigned long long t = 0;
            for (int i = 0; i < kSub; ++i) t += a[i];
            return t;
        };
        if (explicit0 && first == 0) {
            // The explicit round-0 list counted itself; an empty one means
            // the solo part matched every instance.
            live_e[0] = (int64_t)sum(ring[0].live);
            live_p[0] = (int64_t)sum(ring[0].kappa);
            if (live_e[0] == 0) {
                finished = true;
                rounds = 0;
                launched = first;
            }
        }
        // A tail that took over at round t0 ran rounds t0 onwards: the ring
        // holds the rounds before it.
        const bool tail_taken = tail_launched && tail_head[0] != 0;
        if (tail_launched && !tail_taken) tail_missed = true;
        const int ring_end = tail_taken ? std::min(launched, (int)tail_head[0] - 1) : launched;
        for (int r = first; r < ring_end; ++r) {
            const RoundStats &cur = ring[r % lay.ring];
            const RoundStats &nxt = ring[(r + 1) % lay.ring];
            matched_r.push_back((int64_t)sum(cur.matched));
            weight_r.push_back(sum(cur.weight));
            matched_p.push_back((int64_t)sum(cur.mpins));
            const unsigned long long live_next = sum(nxt.live);
            if (live_next == 0) {
                finished = true;
                rounds = r + 1;
                break;
            }
            live_e.push_back((int64_t)live_next);
            live_p.push_back((int64_t)sum(nxt.kappa));
        }
        if (tail_taken) {
            // Rounds t0 .. end - 1 ran in the tail; its record holds their counts.
            const int t0 = (int)tail_head[0] - 1, end = (int)tail_head[1];
            const int nrows = end - t0;
            std::vector<unsigned long long> row(5 * (size_t)std::max(nrows, 0));
            if (nrows > kTailRowsFirst) {
                HGM_TRY(hipMemcpyAsync(row.data(), s.tail + kTailHeader,
                                       sizeof(unsigned long long) * row.size(),
                                       hipMemcpyDeviceToHost, L.stream));
                HGM_TRY(hipStreamSynchronize(L.stream));
            } else if (nrows > 0) {
                std::copy(tail_head.begin() + kTailHeader,
                          tail_head.begin() + kTailHeader + 5 * (size_t)nrows, row.begin());
            }
            for (int j = 0; j < nrows; ++j) {
                if (j > 0) {  // round t0's live counts came from the ring
                    live_e.push_back((int64_t)row[5 * j + 0]);
                    live_p.push_back((int64_t)row[5 * j + 1]);
                }
                matched_r.push_back((int64_t)row[5 * j + 2]);
                weight_r.push_back(row[5 * j + 3]);
                matched_p.push_back((int64_t)row[5 * j + 4]);
            }
            if (tail_head[2] == 1) return HGM_E_ROUND_LIMIT;
            if (tail_head[2]) return HGM_E_HIP;  // the tail's round bound was exceeded
            finished = true;
            rounds = end;
        }
        if (max0_event >= 0 && T.on && max0_event < (int)T.cls.size()) {
            T.cls[max0_event] = ring[0].form == 1 ? HGM_K_SCATTER : HGM_K_VERTEX_MAX;
            max0_event = -1;
        }
        HGM_TRY(T.harvest(finished ? rounds : launched + 1, stats, round_ms));
        if (!finished && o.max_rounds > 0 && launched >= o.max_rounds) return HGM_E_ROUND_LIMIT;
    }

    int64_t tm = 0;
    uint64_t tw = 0;
    for (int r = 0; r < rounds; ++r) {
        tm += matched_r[r];
        tw += weight_r[r];
    }
    if (explicit0 && g.m > 0) {
        // Merge the solo part: its rounds count from each instance's own
        // round 0, like the round kernels' rounds.
        if (solo_head[1]) return HGM_E_ROUND_LIMIT;
        const int sr = (int)solo_head[0];
        const int rows = std::min(sr, lay.solo_rounds);
        std::vector<unsigned long long> row(5 * (size_t)rows);
        if (rows > kSoloRowsFirst) {
            HGM_TRY(hipMemcpyAsync(row.data(), s.solo + kSoloHeader,
                                   sizeof(unsigned long long) * row.size(),
                                   hipMemcpyDeviceToHost, L.stream));
            HGM_TRY(hipStreamSynchronize(L.stream));
        } else if (rows > 0) {
            std::copy(solo_head.begin() + kSoloHeader,
                      solo_head.begin() + kSoloHeader + 5 * (size_t)rows, row.begin());
        }
        const int total = std::max(rounds, sr);
        live_e.resize(std::max<size_t>(live_e.size(), (size_t)total), 0);
        live_p.resize(std::max<size_t>(live_p.size(), (size_t)total), 0);
        matched_r.resize(std::max<size_t>(matched_r.size(), (size_t)total), 0);
        matched_p.resize(std::max<size_t>(matched_p.size(), (size_t)total), 0);
        weight_r.resize(std::max<size_t>(weight_r.size(), (size_t)total), 0);
        for (int r = 0; r < rows; ++r) {
            live_e[r] += (int64_t)row[5 * r + 0];
            live_p[r] += (int64_t)row[5 * r + 1];
            matched_r[r] += (int64_t)row[5 * r + 2];
            weight_r[r] += row[5 * r + 3];
            matched_p[r] += (int64_t)row[5 * r + 4];
        }
        tm += (int64_t)solo_head[3];
        tw += solo_head[4];
        rounds = total;
    }
    if (stats) {
        stats->rounds = rounds;
        for (int r = 0; r < rounds; ++r) {
            if (r < stats->cap) {
                if (stats->live_edges) stats->live_edges[r] = live_e[r];
                if (stats->live_pins) stats->live_pins[r] = live_p[r];
                if (stats->matched_per_round) stats->matched_per_round[r] = matched_r[r];
                if (stats->matched_pins) stats->matched_pins[r] = matched_p[r];
                if (stats->round_ms) stats->round_ms[r] = r < (int)round_ms.size() ? round_ms[r] : 0.f;
            }
        }
        stats->matched = tm;
        stats->weight = tw;
    }
    return HGM_OK;
}


// Workspace of hgm_match_noalloc: one array per GPU in the library's device
// memory, held until the process ends.  In host code `scratch` names a host
// stand-in, not the device array, so the array is only ever used through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxDevices];  // zero-initialised (static storage)
std::mutex g_scratch_mu;

// Device address of the current device's scratch array (looked up once per
// device, with that device current), or NULL on a HIP error.
void *scratch_address() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (p) return p;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev].store(p, std::memory_order_release);
    return p;
}

// Shared body of hgm_match and hgm_match_noalloc.
int match_one(const hgm_csr *gin, uint32_t seed, uint32_t *matched_bits, void *workspace,
              size_t ws_bytes, const hgm_opts *opts, void *stream, hgm_stats *stats) {
    Opts o;
    int rc = resolve_opts(opts, &o);
    if (rc != HGM_OK) return rc;
    rc = check_graph(gin, o);
    if (rc != HGM_OK) return rc;
    bind_graph(&o, gin);
    if (gin->m > 0 && !matched_bits) return HGM_E_ARG;
    if (stats && stats->cap < 0) return HGM_E_ARG;
    const Layout lay = make_layout(gin->n, gin->m, gin->kappa, o);
    if (!workspace) return HGM_E_ARG;
    if (ws_bytes < lay.total) return HGM_E_SIZE;
    if (((uintptr_t)workspace & 255) != 0) return HGM_E_ARG;

    Graph g;
    memset(&g, 0, sizeof(g));
    g.n = gin->n;
    g.m = gin->m;
    g.kappa = gin->kappa;
    g.words = ((int64_t)gin->m + 31) / 32;
    g.pairs = o.pairs ? 1 : 0;
    g.e_off = o.pairs ? nullptr : gin->e_off;
    g.e_pins = gin->e_pins;
    g.v_off = gin->v_off;
    g.v_edges = gin->v_edges;
    g.w = gin->w;
    const State s = carve(workspace, lay, o);
    Launch L;
    L.grid = device_cus() * o.blocks_per_cu;
    L.stream = (hipStream_t)stream;
    if (L.grid <= 0) return HGM_E_HIP;
    return run_rounds(g, o, lay, s, L, seed, matched_bits, stats, nullptr);
}

}  // namespace

extern "C" {

int hgm_version(void) { return 400; }

#ifndef HGM_SOURCE_DIGEST
#define HGM_SOURCE_DIGEST "unknown"
#endif
const char *hgm_source_digest(void) { return HGM_SOURCE_DIGEST; }

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
    bind_graph(&o, g);
    if (g->n < 0 || g->m < 0 || g->kappa < 0 || g->kappa >= ((int64_t)1 << 31)) return 0;
    return make_layout(g->n, g->m, g->kappa, o).total;
}

int hgm_match(const hgm_csr *gin, uint32_t seed, uint32_t *matched_bits, void *workspace,
              size_t ws_bytes, const hgm_opts *opts, void *stream, hgm_stats *stats) {
    return match_one(gin, seed, matched_bits, workspace, ws_bytes, opts, stream, stats);
}

size_t hgm_noalloc_max_bytes(void) { return kScratchBytes; }

int hgm_match_noalloc(const hgm_csr *gin, uint32_t seed, uint32_t *matched_bits,
                      const hgm_opts *opts, void *stream, hgm_stats *stats) {
    // Per-kernel timing creates HIP events, which this entry point avoids.
    if (stats && stats->timing) return HGM_E_ARG;
    const size_t need = hgm_workspace_size(gin, opts);
    if (need == 0) {  // invalid sizes or options: the checks of hgm_match report which
        Opts o;
        int rc = resolve_opts(opts, &o);
        if (rc != HGM_OK) return rc;
        rc = check_graph(gin, o);
        return rc != HGM_OK ? rc : HGM_E_ARG;
    }
    if (need > kScratchBytes) return HGM_E_SIZE;
    void *ws = scratch_address();
    if (!ws) return HGM_E_HIP;
    return match_one(gin, seed, matched_bits, ws, kScratchBytes, opts, stream, stats);
}

size_t hgm_batch_workspace_size(const hgm_batch *b, const hgm_opts *opts) {
    Opts o;
    if (resolve_opts(opts, &o) != HGM_OK || check_batch(b, o) != HGM_OK) return 0;
    bind_batch(&o, b);
    return make_layout(b->n_total, b->m_total, b->kappa_total, o, true).total;
}

int hgm_match_batch(const hgm_batch *b, uint32_t *matched_bits, void *workspace, size_t ws_bytes,
                    const hgm_opts *opts, void *stream, hgm_stats *stats) {
    Opts o;
    int rc = resolve_opts(opts, &o);
    if (rc != HGM_OK) return rc;
    rc = check_batch(b, o);
    if (rc != HGM_OK) return rc;
    bind_batch(&o, b);
    if (b->m_total > 0 && !matched_bits) return HGM_E_ARG;
    if (stats && stats->cap < 0) return HGM_E_ARG;
    const Layout lay = make_layout(b->n_total, b->m_total, b->kappa_total, o, true);
    if (!workspace) return HGM_E_ARG;
    if (ws_bytes < lay.total) return HGM_E_SIZE;
    if (((uintptr_t)workspace & 255) != 0) return HGM_E_ARG;

    const State s = carve(workspace, lay, o);
    char *base = (char *)workspace;
    BatchIn in;
    in.count = b->count;
    in.v_base = b->v_base;
    in.e_base = b->e_base;
    in.pin_base = b->pin_base;
    in.word_base = b->word_base;
    in.e_off = b->e_off;
    in.v_off = o.have_vertex_side ? b->v_off : nullptr;
    in.seeds = b->seeds;
    in.reseed = o.reseed ? 1 : 0;
    in.goff = (int32_t *)(base + lay.goff);
    in.vbase = (int32_t *)(base + lay.vbase);
    in.bitoff = (int32_t *)(base + lay.bitoff);
    in.gvoff = o.have_vertex_side ? (int32_t *)(base + lay.gvoff) : nullptr;
    in.ebase = o.have_vertex_side ? (int32_t *)(base + lay.ebase) : nullptr;

    Graph g;
    memset(&g, 0, sizeof(g));
    g.n = (int32_t)b->n_total;
    g.m = (int32_t)b->m_total;
    g.kappa = b->kappa_total;
    g.words = b->words_total;
    g.e_off = in.goff;
    g.e_pins = b->e_pins;
    g.v_off = in.gvoff;
    g.v_edges = b->v_edges;
    g.w = b->w;
    g.vbase = in.vbase;
    g.bitoff = in.bitoff;
    g.ebase = in.ebase;
    Launch L;
    L.grid = device_cus() * o.blocks_per_cu;
    L.stream = (hipStream_t)stream;
    if (L.grid <= 0) return HGM_E_HIP;
    SoloArgs sa;
    memset(&sa, 0, sizeof(sa));
    if (s.explicit0) {
        sa.count = b->count;
        sa.v_base = b->v_base;
        sa.e_base = b->e_base;
        sa.pin_base = b->pin_base;
        sa.word_base = b->word_base;
        sa.max_kappa = o.solo_max_kappa ? o.solo_max_kappa : solo_auto_bound(b->kappa_total);
        sa.lds_bytes = solo_lds_bytes();
        if (sa.lds_bytes <= 0) return HGM_E_HIP;
        sa.one_tile = solo_verts_for(sa.lds_bytes, 1);
        sa.max_verts = solo_verts_for(sa.lds_bytes, kSoloMaxTiles);
        sa.max_rounds = o.max_rounds;
    }
    return run_rounds(g, o, lay, s, L, 0, matched_bits, stats, &in, &sa);
}

int hgm_solo_lds_vertices(void) {
    const int bytes = solo_lds_bytes();
    return bytes > 0 ? solo_verts_for(bytes, 1) : 0;
}

}  // extern "C"
