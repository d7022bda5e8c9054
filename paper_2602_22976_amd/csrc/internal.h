// Internal interface between the round kernels (kernels.hip) and the host
// driver (api.hip).  Not installed; the public interface is include/hgm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hgm {

constexpr int kBlock = 256;  // threads per workgroup = edges (or vertices) per chunk
constexpr int kSub = 64;     // counters are spread over kSub addresses (one per 64 blocks)
constexpr int kHubPiece = 8192;  // incidences of a hub vertex reduced by one workgroup

__host__ __device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) {
    return (x << r) | (x >> (32 - r));
}

// MurmurHash3_x86_32 (Appleby) of the four little-endian bytes of `id`:
// one body block, no tail, length 4, then the fmix32 finaliser.  Every step
// is invertible on 32-bit words, so for a fixed seed it is a bijection of id.
// Edge priorities are H(seed, e); when the order is drawn afresh every round,
// round r uses the seed H(seed, r) (round_seed).
__host__ __device__ __forceinline__ uint32_t priority_hash(uint32_t seed, uint32_t id) {
    uint32_t k = id * 0xcc9e2d51u;
    k = rotl32(k, 15);
    k *= 0x1b873593u;
    uint32_t h = seed ^ k;
    h = rotl32(h, 13);
    h = h * 5u + 0xe6546b64u;
    h ^= 4u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__host__ __device__ __forceinline__ uint32_t round_seed(uint32_t seed, int round) {
    return priority_hash(seed, (uint32_t)round);
}

// Per-round counters, in a small device ring indexed by round % ring.  Every
// field is split into kSub partial sums (block b adds into entry b % kSub)
// so that no single address takes one atomic per workgroup; the host sums.
struct RoundStats {
    unsigned long long live[kSub];     // live edges at the start of the round (|L_r|)
    unsigned long long kappa[kSub];    // sum of their sizes (kappa_r)
    unsigned long long matched[kSub];  // edges matched in the round
    unsigned long long weight[kSub];   // their total weight
    unsigned long long mpins[kSub];    // their total size
    unsigned long long form;           // round 0 only: 1 edge-centric, 2 vertex-centric maximum
    unsigned long long bin_overflow;   // binned maximum: a bin received more records than
                                       // its vertices' degrees allow (v_off is not the
                                       // transpose of e_pins); those records were dropped
};

// The hypergraph as the kernels see it.  A batch of independent instances is
// matched as their disjoint union: e_off / v_off are then global offsets built
// by k_batch_setup, while e_pins / v_edges keep the caller's instance-local
// ids, turned global by adding the per-edge vertex base / per-vertex edge
// base.  For one instance the three base arrays are NULL (all zero).
struct Graph {
    int32_t n, m;
    int64_t kappa;
    int64_t words;           // bitmap words
    int32_t pairs;           // every edge has two pins at e_pins[2e], e_pins[2e + 1]; e_off unused
    const int32_t *e_off;
    const int32_t *e_pins;
    const int32_t *v_off;
    const int32_t *v_edges;
    const uint32_t *w;
    const int32_t *vbase;    // [m] added to the pins of edge e (batch)
    const int32_t *bitoff;   // [m] bitmap bit of edge e is e + bitoff[e] (batch)
    const int32_t *ebase;    // [n] added to the incident edges of vertex v (batch)
};

// Caller's batch arrays (device), for k_batch_setup.
struct BatchIn {
    int32_t count;
    const int64_t *v_base, *e_base, *pin_base, *word_base;  // [count + 1]
    const int32_t *e_off;     // [m_total + count] local offsets, instance i at e_base[i] + i
    const int32_t *v_off;     // [n_total + count] local offsets, instance i at v_base[i] + i
    const uint32_t *seeds;    // [count]
    int32_t reseed;           // priorities redrawn every round: keys of round 0 use
                              // H(seed_i, 0) and eseed keeps seed_i and the local id
    int32_t *goff;            // out [m_total + 1]
    int32_t *vbase;           // out [m_total]
    int32_t *bitoff;          // out [m_total]
    int32_t *gvoff;           // out [n_total + 1] (NULL: no vertex side)
    int32_t *ebase;           // out [n_total]
};

// Device state of one hgm_match call, carved out of the caller's workspace.
//
// Live edges are kept per workgroup: edge kernels run exactly `grid`
// workgroups, and workgroup b owns the edges with ids in
// [b * region, (b + 1) * region).  Its live edges of round r sit in
// list[r & 1][b * region ...] with count cnt[r & 1][b]; round 0 is the
// identity.  Compaction is therefore local to a workgroup and needs no
// global atomic, and an edge stays with the same workgroup for the whole run.
struct State {
    uint64_t *key;      // [m] batch only: packed key w<<32 | H(seed_i, local id); NULL for
                        // one instance, whose keys are rebuilt from w and the round's seed
    uint64_t *eseed;    // [m] batch with priorities redrawn every round: seed_i << 32 |
                        // local id, from which round r's key is rebuilt (NULL otherwise)
    uint64_t *best[2];  // [n] per-vertex maximum live key, double-buffered by round parity
    uint8_t *done;      // [n] vertex is a pin of a matched edge
    int32_t *list[2];   // [grid * region] live edges per workgroup region
    int32_t *cnt[2];    // [grid] live edges per region
    // Edge records beside list[] (same index), written by the retire pass for
    // every survivor so that the next kernels read them with the id instead
    // of gathering through it.  Offset layout: rec_a = first pin offset,
    // rec_b = pin count, rec_c = first pin (vertex id, batch base added).
    // Pair layout: rec_a, rec_b = the two pins.  rec_key = the key of the
    // list's round; rec_vb = the edge's vertex base (batch only).
    int32_t *rec_a[2], *rec_b[2], *rec_c[2], *rec_vb[2];
    uint64_t *rec_key[2];
    RoundStats *stats;  // [ring]
    int32_t ring;
    int32_t grid;       // edge-kernel workgroups
    int32_t region;     // edge ids (and list capacity) per workgroup, multiple of kBlock
    int32_t *err;       // [1] validation error flag
    // Vertex-centric (CREW) extras
    uint64_t *live_key; // [m] key while live, 0 once matched or retired (CREW variant);
                        // with priorities redrawn every round w << 32 | 1 while live
                        // (a liveness mark that keeps the weight)
    int2 *pieces;       // [piece_cap] (hub vertex, piece index): the incidence list of a
                        // vertex of degree > hub threshold is cut into kHubPiece pieces
    int32_t *piece_count;  // [1]
    unsigned long long *hot;  // [kSub] incidences on vertices of degree >= hot_degree
    uint32_t *wrange;   // [2 * kSub] smallest and largest weight (kInitWeightRange, or
                        // AUTO's round-0 edge kernel when the vertex form runs): slot
                        // k holds workgroups b = k mod kSub, min at 2k, max at 2k + 1
    int32_t *vedges[2]; // [kappa] live incident edges of each vertex (global ids) at the
                        // front of its v_off segment, compacted by the vertex pass of
                        // rounds with parity 0 / 1 (CREW variant)
    int32_t *vlen[2];   // [n] their counts
    int32_t piece_cap;
    int32_t hub_threshold;
    int32_t hot_degree;  // vertices of at least this degree are hot (AUTO's round-0 form)
    uint32_t *vbits;    // [ceil(kappa/32)] validation: edge-side incidences seen
    // Batch with a solo part: round 0's live list is not the identity but an
    // explicit list[0] / cnt[0] with records, holding only the edges of the
    // instances the round kernels match (the others ran in k_solo).
    int32_t explicit0;
    unsigned long long *solo;  // [kSoloHeader + 5 * solo_rounds] per-round sums of the solo
                               // instances (see SoloArgs); NULL without a solo part
    int32_t solo_rounds;       // rows of per-round sums
    // Tail of one instance (k_tail): a compact live list, double-buffered,
    // with each edge's pin offset and count (pair layout: its two pins) and
    // key; and the tail's record (see kTailHeader).  tail_cap = 0: no tail.
    int32_t *tail_e[2], *tail_a[2], *tail_b[2];
    uint64_t *tail_key[2];
    unsigned long long *tail;
    int32_t tail_cap;          // live edges the tail takes at most
    int64_t tail_pins;         // it takes over a round with at most this many live pins
    // Binned maximum (one instance, offset layout, vertex side given): the
    // retire pass writes each surviving non-hub pin's record (pin's index in
    // its bin, key) to the bin of 2^bin_rb consecutive vertices holding it,
    // and k_bin_max reduces every bin in LDS.  Bin j's records sit at
    // v_off[j << bin_rb] + [0, bin_cursor[j]): the bin's vertices' degrees
    // bound its records in any round.  bin_nb = 0: no bins.
    uint16_t *bin_v;           // [kappa]
    uint64_t *bin_key;         // [kappa]
    uint32_t *bin_cursor;      // [bin_nb] records written, zero between passes
    int32_t bin_rb, bin_nb;
    int32_t bin_auto;          // bins only where round 0 took the vertex form (the
                               // degree profile in `hot`); 0: in every binned round
};

constexpr int kBinMaxBins = 1024;     // bins of one instance at most
constexpr int kBinMinShift = 10, kBinMaxShift = 14;  // 2^14 keys = 128 KB of LDS
constexpr int kBinThreads = 1024;     // workgroup of k_bin_max

// Tail record: word 0 = 1 + the round the tail took over at (0: not taken),
// word 1 = the rounds of the whole matching when it finished, word 2 =
// 1 when max_rounds stopped it with live edges (2: it ran more rounds than it
// had live edges, which a correct maximum never does); then row j holds live
// edges, live pins, matched edges, their weight and their pins of round
// (taken round + j).
constexpr int kTailHeader = 8;
constexpr int kTailThreads = 1024;

// Solo part of a batch: instances with at most max_kappa pins and at most
// max_verts vertices are matched whole by one workgroup each (k_solo), every
// round inside the workgroup.  Their done flags are a bitmask in LDS, and
// best is kept in LDS in tiles of vertices: instances with at most one_tile
// vertices need one tile, larger ones (up to kSoloMaxTiles tiles) form and
// test each round's maximum tile by tile.  Per-round sums go to State::solo:
// header word 0 = most rounds of any solo instance, word 1 = nonzero when an
// instance reached max_rounds with live edges, word 2 = the work counter,
// words 3 and 4 = matched edges and their weight over all rounds; then row r
// holds live edges, live pins, matched edges, their weight and their pins of
// round r summed over the solo instances (rows beyond solo_rounds are not
// recorded; the host never asks for them).
constexpr int kSoloHeader = 8;
constexpr int kSoloThreads = 1024;
constexpr int kSoloStaticLds = 24 * 1024;  // bound on k_solo's own shared variables
constexpr int kSoloMaxTiles = 8;
struct SoloArgs {
    int32_t count;
    const int64_t *v_base, *e_base, *pin_base, *word_base;  // the caller's [count + 1]
    int64_t max_kappa;
    int32_t max_verts;
    int32_t one_tile;
    int32_t lds_bytes;   // dynamic LDS of a workgroup: done bitmask, then best tiles
    int32_t max_rounds;  // 0 = no limit
};

// Whether instance i of a batch (n_i vertices, kappa_i pins) is matched by k_solo.
__host__ __device__ __forceinline__ bool solo_instance(int64_t n_i, int64_t kappa_i,
                                                       const SoloArgs &a) {
    return kappa_i <= a.max_kappa && n_i <= a.max_verts;
}

struct Launch {
    int grid;            // persistent workgroup count for vertex / setup kernels
    hipStream_t stream;
};

// init_flags: which optional setup k_init performs.
constexpr int kInitLiveKey = 1;  // copy keys to live_key (CREW variant)
constexpr int kInitHubs = 2;     // cut high-degree vertices into pieces (any CREW round)
constexpr int kInitWeightRange = 4;  // smallest and largest weight (CREW round-0 vertex pass,
                                     // one instance: equal weights need no gather)
constexpr int kInitLiveMark = 8;     // with kInitLiveKey: live_key = w << 32 | 1 (priorities
                                     // redrawn every round)
// `kseed` arguments: the priority seed of the round the kernel works on
// (the call's seed, or round_seed(seed, r) when the order is redrawn);
// `rekey`: nonzero when the order is redrawn every round.
hipError_t launch_init(const Launch &L, const Graph &g, uint32_t seed, const State &s,
                       uint32_t *bits, int init_flags);
hipError_t launch_batch_setup(const Launch &L, const Graph &g, const BatchIn &b, const State &s);
// Solo part of a batch, then the explicit round-0 list of the other instances.
hipError_t launch_solo(const Launch &L, const Graph &g, const State &s, const SoloArgs &a,
                       uint32_t *bits, int rekey, int workgroups);
hipError_t launch_live0(const Launch &L, const Graph &g, const State &s, const SoloArgs &a);
hipError_t launch_validate(const Launch &L, const Graph &g, const State &s, int check_dual);
hipError_t launch_scatter(const Launch &L, const Graph &g, const State &s, uint32_t kseed);
// binned (CRCW form, one instance, offset layout, s.bin_nb > 0): the next
// round's maximum by bins (k_retire_bin, then k_bin_max) instead of atomics.
hipError_t launch_retire(const Launch &L, const Graph &g, const State &s, int round, int scatter,
                         uint32_t kseed, int rekey, int binned = 0);
hipError_t launch_vertex_max(const Launch &L, const Graph &g, const State &s, int round,
                             uint32_t kseed, int rekey);
// Round-0 maximum in the form chosen from the degree profile (AUTO): two
// launches, of which the one not chosen returns at once.
hipError_t launch_max0(const Launch &L, const Graph &g, const State &s, uint32_t seed);
// How the test clears the next round's maximum buffer (see k_test).
constexpr int kClearNone = 0, kClearAll = 1, kClearPins = 2;
hipError_t launch_test(const Launch &L, const Graph &g, const State &s, int round, int clear,
                       uint32_t *bits, uint32_t kseed);
// One workgroup checks round `round`'s live counts and, when they are within
// the tail's bounds, runs every remaining round of the instance (one
// instance, offset or pair layout; seed and reseed as for the other kernels).
hipError_t launch_tail(const Launch &L, const Graph &g, const State &s, int round,
                       uint32_t *bits, uint32_t seed, int reseed, int max_rounds);

}  // namespace hgm
