// Round kernels of iterated local-max hypergraph matching for gfx950.
//
// One round of the method (paper, Section 4.1 and Algorithms 1/2):
//   max    every vertex v takes best[v] = max key over its live incident edges
//   test   a live edge e whose key equals best[v] at every pin v is matched;
//          its pins are marked done
//   retire every live edge with a done pin leaves the live set (soft delete)
// Keys: key(e) = w(e) << 32 | H(seed, e), with H = MurmurHash3_x86_32 of e's
// little-endian bytes; H is a bijection, so keys are distinct.  The seed is
// the call's in every round (fixed order), or round_seed(seed, r) in round r
// when the order is redrawn every round; kernels take it as `kseed`.
//
// Work layout.  All kernels are persistent (grid = a few workgroups per CU)
// and walk their input in chunks of kBlock items (live edges or vertices).
// Inside a chunk the items' incidence lists are flattened: an exclusive scan of
// the sizes gives each item's start, and the chunk's incidences are spread
// over all lanes, kBlock at a time, each lane finding its item by binary
// search over the starts in LDS.  Load balance is thus independent of the
// size distribution (Zipf sizes up to 64 cost no more lanes than they use),
// and consecutive lanes read consecutive pins.
//
// Edge kernels run exactly s.grid workgroups; workgroup b owns the edge ids
// [b * region, (b + 1) * region) for the whole run and keeps its live ones in
// its own region of list[r & 1] (round 0: the identity).  Counters of round r
// go to stats[r % ring], spread over kSub addresses.  best[] is
// double-buffered by round parity so that the test of round r can clear the
// buffer round r+1 will fill.
#include <atomic>

#include "internal.h"

namespace hgm {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

// Key of edge e in a round whose priority seed is kseed.  A batch stores its
// keys (each instance has its own seed and local ids); one instance rebuilds
// them from the 4-byte weight, half the bytes of a stored key.
// kB (here and below): the kernels run on a batch (stored keys, per-edge
// vertex bases, bitmap offsets) rather than one instance; each kernel is
// instantiated for both and the host launches the one that applies.
template <bool kB>
__device__ __forceinline__ uint64_t edge_key(const Graph &g, const State &s, uint32_t kseed,
                                             int e) {
    if constexpr (kB) return s.key[e];
    return ((uint64_t)g.w[e] << 32) | priority_hash(kseed, (uint32_t)e);
}

// Key of edge e in round `round` when priorities are redrawn every round.
// One instance: kseed is the round's seed H(seed, round), derived on the
// host.  A batch: each instance has its own seed, so the round seed
// H(seed_i, round) is derived per edge from the seed and local id that the
// batch setup kept.
template <bool kB>
__device__ __forceinline__ uint64_t round_key(const Graph &g, const State &s, uint32_t kseed,
                                              int round, int e) {
    if constexpr (kB) {
        const uint64_t sl = s.eseed[e];
        const uint32_t rs = round_seed((uint32_t)(sl >> 32), round);
        return ((uint64_t)g.w[e] << 32) | priority_hash(rs, (uint32_t)sl);
    }
    return edge_key<false>(g, s, kseed, e);
}

// v plus the value DPP control kCtrl reads for this lane (0 where it reads
// none or the row is masked off).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_add(int v) {
    return v + __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, false);
}

// Inclusive prefix sum over a wave with DPP lane moves (VALU, no LDS
// traffic): row shifts by 1, 2, 4, 8 sum each row of 16 lanes; lane 15 of
// each row then adds into rows 1 and 3, and lane 31 into rows 2 and 3.
__device__ __forceinline__ int wave_inclusive_sum(int v) {
    v = dpp_add<0x111, 0xF>(v);  // row_shr:1
    v = dpp_add<0x112, 0xF>(v);  // row_shr:2
    v = dpp_add<0x114, 0xF>(v);  // row_shr:4
    v = dpp_add<0x118, 0xF>(v);  // row_shr:8
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Segmented inclusive max-scan over a wave with DPP lane moves (VALU), not
// ds_bpermute shuffles, which go through the LDS pipe that the vertex pass
// already keeps busy with its item searches.  Segments are runs of equal j
// (contiguous).  Row shifts by 1, 2, 4, 8 scan each row of 16 lanes; then
// lane 15 of each row is broadcast into rows 1 and 3, and lane 31 into rows
// 2 and 3.  A lane takes the value it reads only when it reads from its own
// segment; lanes with no source keep j = -2, which equals no j.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_max_dpp(uint64_t &k, int j) {
    const int yj = __builtin_amdgcn_update_dpp(-2, j, kCtrl, kRowMask, 0xF, false);
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)k, kCtrl, kRowMask, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k >> 32), kCtrl,
                                                              kRowMask, 0xF, false);
    const uint64_t y = ((uint64_t)hi << 32) | lo;
    if (yj == j && y > k) k = y;
}

constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114,
              kDppRowShr8 = 0x118, kDppBcast15 = 0x142, kDppBcast31 = 0x143,
              kDppWaveShl1 = 0x130;

__device__ __forceinline__ uint64_t wave_segmented_max(uint64_t k, int j) {
    seg_max_dpp<kDppRowShr1, 0xF>(k, j);
    seg_max_dpp<kDppRowShr2, 0xF>(k, j);
    seg_max_dpp<kDppRowShr4, 0xF>(k, j);
    seg_max_dpp<kDppRowShr8, 0xF>(k, j);
    seg_max_dpp<kDppBcast15, 0xA>(k, j);
    seg_max_dpp<kDppBcast31, 0xC>(k, j);
    return k;
}

// j of the next lane (lane 63: -2).
__device__ __forceinline__ int next_lane_j(int j) {
    return __builtin_amdgcn_update_dpp(-2, j, kDppWaveShl1, 0xF, 0xF, false);
}

// Exclusive block-wide prefix sum of v; *total receives the block sum.
// Contains two barriers; every thread of the block must call it.
__device__ __forceinline__ int block_exclusive_sum(int v, int *wave_tmp, int *total) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    int incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) wave_tmp[wid] = incl;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        int x = wave_tmp[i];
        off += (i < wid) ? x : 0;
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return off + incl - v;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *tmp) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) tmp[wid] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += tmp[i];
    __syncthreads();
    return t;
}

// The work item (edge region or run of vertex chunks) of workgroup b among
// `grid`.  The dispatcher deals workgroups to the chip's 8 XCDs round-robin
// (b on XCD b % 8), and each XCD has its own L2: mapping each XCD's
// workgroups to one contiguous share of the items keeps neighbouring items,
// e.g. the edges and vertices of one instance of a batch, on one L2 instead
// of all eight.  A bijection of [0, grid).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int grid) {
    const int x = b % kXcds, q = b / kXcds;
    const int per = grid / kXcds, rem = grid % kXcds;
    return x * per + (x < rem ? x : rem) + q;
}

// Largest j in [0, kBlock) with start[j] <= t (start non-decreasing, start[0] = 0).
__device__ __forceinline__ int find_item(const int *start, int t) {
    int j = 0;
#pragma unroll
    for (int step = kBlock / 2; step > 0; step >>= 1)
        if (start[j + step] <= t) j += step;
    return j;
}

// Read of a best[] entry that other workgroups raise with atomics during the
// same pass.  Workgroup scope lets the load hit in L2 (an agent-scope load
// bypasses it on this chip); the value may be stale, but best[] only grows
// within a pass, so a stale value is a lower bound and skipping the atomic
// when it is already >= the key is still exact.
__device__ __forceinline__ uint64_t load_lower_bound(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void atomic_max_u64(uint64_t *p, uint64_t v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Shared-memory layout of one chunk of items.
struct ChunkLds {
    int start[kBlock];        // exclusive scan of incidence counts
    int base[kBlock];         // offset of each item's list in the pin / edge array
    uint64_t key[kBlock];     // edge keys (edge chunks) or running maxima (vertex chunks)
    int flag[kBlock];         // per-item flag (failed test / retired)
    int vb[kBlock];           // per-item id base (batch: vertex base of an edge, edge base of a vertex)
    int wave_tmp[kWaves];
    unsigned long long sum_tmp[kWaves];
};

// Incidences a lane visits per step of a flattened loop.  Their pin loads and
// the gathers that follow are independent, so a lane keeps this many memory
// requests in flight instead of one.
constexpr int kUnroll = 4;

// The kUnroll incidences t0, t0 + kBlock, ... of the current chunk: item
// index j (-1 past the end) and pin.
template <bool kB>
__device__ __forceinline__ void chunk_pins(const ChunkLds &L, const int32_t *e_pins, int total,
                                           int t0, int (&j)[kUnroll], int (&pin)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int t = t0 + u * kBlock;
        j[u] = t < total ? find_item(L.start, t) : -1;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
        pin[u] = j[u] >= 0 ? e_pins[L.base[j[u]] + (t0 + u * kBlock - L.start[j[u]])] +
                                 (kB ? L.vb[j[u]] : 0)
                           : 0;
}

// Raises best[pin] to the chunk items' keys over a flattened loop.  The
// plain read first skips the atomic when the slot already holds a larger key
// (best only grows during the pass, so a stale read is merely cautious).
// One incidence per lane and step: issuing more reads before the atomics
// makes more of them see stale values and turns filtered reads into atomics,
// which cost far more on this hardware than the latency saved.
template <bool kB>
__device__ __forceinline__ void scatter_chunk(const ChunkLds &L, const int32_t *e_pins, int total,
                                              uint64_t *best) {
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int j = find_item(L.start, t);
        const int pin = e_pins[L.base[j] + (t - L.start[j])] + (kB ? L.vb[j] : 0);
        const uint64_t k = L.key[j];
        if (load_lower_bound(&best[pin]) < k) atomic_max_u64(&best[pin], k);
    }
}

// Per-workgroup table of hub vertices (degree above the hub threshold, as
// listed by the hub pieces) for the round-0 edge scatter.  Every workgroup
// meets the few hubs in a large share of its incidences, and device atomics
// on one address serialise, so a hub's pins are reduced in LDS for the
// workgroup's whole region and pushed to best[] once at the end.  Open
// addressing with linear probing; at most half the slots are filled, so a
// probe always reaches the hub or an empty slot.
constexpr int kHubSlotBits = 10;
constexpr int kHubSlots = 1 << kHubSlotBits;
constexpr int kHubTableMax = kHubSlots / 2;

struct HubTable {
    int id[kHubSlots];                 // hub vertex, -1 = empty
    unsigned long long mx[kHubSlots];  // the workgroup's largest key at that hub
    int count;
};

__device__ __forceinline__ int hub_home(int v) {
    return (int)(((uint32_t)v * 0x9E3779B1u) >> (32 - kHubSlotBits));
}

// Slot of v, or -1 when v is not in the table.
__device__ __forceinline__ int hub_find(const HubTable &H, int v) {
    int h = hub_home(v);
    for (;;) {
        const int id = H.id[h];
        if (id == v) return h;
        if (id < 0) return -1;
        h = (h + 1) & (kHubSlots - 1);
    }
}

// Fills the table from the hub pieces (one piece with index 0 per hub).
// Hubs beyond kHubTableMax stay out and take the global path.
__device__ void hub_table_build(HubTable &H, const State &s) {
    for (int i = threadIdx.x; i < kHubSlots; i += kBlock) {
        H.id[i] = -1;
        H.mx[i] = 0;
    }
    if (threadIdx.x == 0) H.count = 0;
    __syncthreads();
    const int np = min(*s.piece_count, s.piece_cap);
    for (int q = threadIdx.x; q < np; q += kBlock) {
        const int2 pc = s.pieces[q];
        if (pc.y != 0 || atomicAdd(&H.count, 1) >= kHubTableMax) continue;
        int h = hub_home(pc.x);
        while (atomicCAS(&H.id[h], -1, pc.x) != -1) h = (h + 1) & (kHubSlots - 1);
    }
    __syncthreads();
}

// scatter_chunk with hub pins reduced in the table.
template <bool kB>
__device__ __forceinline__ void scatter_chunk_hubs(const ChunkLds &L, const int32_t *e_pins,
                                                   int total, uint64_t *best, HubTable &H) {
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int j = find_item(L.start, t);
        const int pin = e_pins[L.base[j] + (t - L.start[j])] + (kB ? L.vb[j] : 0);
        const uint64_t k = L.key[j];
        const int h = hub_find(H, pin);
        if (h >= 0) {
            if (H.mx[h] < k) atomicMax(&H.mx[h], (unsigned long long)k);
        } else if (load_lower_bound(&best[pin]) < k) {
            atomic_max_u64(&best[pin], k);
        }
    }
}

// Graphs (every edge has two pins, stored as e_pins[2e], e_pins[2e + 1]):
// one lane per edge reads both pins with one 8-byte load, and no chunk of
// incidences needs flattening.
__device__ __forceinline__ int2 pair_pins(const Graph &g, int e) {
    return reinterpret_cast<const int2 *>(g.e_pins)[e];
}

__device__ __forceinline__ void scatter_pair(uint64_t *best, int2 p, uint64_t k) {
    const uint64_t b0 = load_lower_bound(&best[p.x]);
    const uint64_t b1 = load_lower_bound(&best[p.y]);
    if (b0 < k) atomic_max_u64(&best[p.x], k);
    if (b1 < k) atomic_max_u64(&best[p.y], k);
}

// ---------------------------------------------------------------------------
// Prologue (one workgroup): round counters, error flag, hub piece counter.
__global__ void __launch_bounds__(kBlock) k_prologue(Graph g, State s) {
    unsigned long long *st = (unsigned long long *)s.stats;
    const int words = s.ring * (int)(sizeof(RoundStats) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < words; i += blockDim.x) st[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && !s.explicit0) {  // an explicit round-0 list counts itself
        s.stats[0].live[0] = (unsigned long long)g.m;
        s.stats[0].kappa[0] = g.m == 0 ? 0ull
                              : g.pairs ? 2ull * (unsigned long long)g.m
                                        : (unsigned long long)g.e_off[g.m];
    }
    if (threadIdx.x == 0) {
        *s.err = 0;
        *s.piece_count = 0;
    }
    if (s.solo && threadIdx.x < kSoloHeader) s.solo[threadIdx.x] = 0;
    if (s.tail && threadIdx.x < kTailHeader) s.tail[threadIdx.x] = 0;
    for (int j = threadIdx.x; j < s.bin_nb; j += blockDim.x) s.bin_cursor[j] = 0;
    if (threadIdx.x < kSub) {
        s.hot[threadIdx.x] = 0;
        s.wrange[2 * threadIdx.x] = 0xFFFFFFFFu;
        s.wrange[2 * threadIdx.x + 1] = 0;
    }
}

// Smallest and largest weight into wrange's kSub slots (the whole grid
// takes part; slot k collects workgroups b = k mod kSub).
__device__ void reduce_weight_range(const Graph &g, const State &s) {
    __shared__ uint32_t wlo, whi;
    uint32_t wmin = 0xFFFFFFFFu, wmax = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // Four independent loads per step: a loop that consumes each load
    // before issuing the next waits one memory latency per step.
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < g.m; i += 4 * stride) {
        const uint32_t a = g.w[i], b = g.w[i + stride], c = g.w[i + 2 * stride],
                       d = g.w[i + 3 * stride];
        const uint32_t lo = min(min(a, b), min(c, d)), hi = max(max(a, b), max(c, d));
        wmin = lo < wmin ? lo : wmin;
        wmax = hi > wmax ? hi : wmax;
    }
    for (; i < g.m; i += stride) {
        const uint32_t wi = g.w[i];
        wmin = wi < wmin ? wi : wmin;
        wmax = wi > wmax ? wi : wmax;
    }
    if (threadIdx.x == 0) {
        wlo = 0xFFFFFFFFu;
        whi = 0;
    }
    __syncthreads();
    atomicMin(&wlo, wmin);
    atomicMax(&whi, wmax);
    __syncthreads();
    if (threadIdx.x == 0 && whi >= wlo) {  // spread over kSub slots: atomics on one
        const int k = blockIdx.x % kSub;     // address serialise
        atomicMin(&s.wrange[2 * k], wlo);
        atomicMax(&s.wrange[2 * k + 1], whi);
    }
}

// Setup: cleared per-vertex state and bitmap; optionally the CREW live keys,
// the pieces of high-degree vertices and the weight range.
__global__ void __launch_bounds__(kBlock) k_init(Graph g, uint32_t seed, State s, uint32_t *bits,
                                                 int flags) {
    __shared__ unsigned long long sum_tmp[kWaves];
    unsigned long long hot = 0;
    const int64_t words = g.words;
    const int64_t edges = (flags & kInitLiveKey) ? g.m : 0;  // edge-indexed work: live keys only
    const int64_t span = edges > g.n ? edges : g.n;
    const int64_t solo_words = s.solo ? 5 * (int64_t)s.solo_rounds : 0;
    const int64_t top0 = span > words ? span : words;
    const int64_t top = top0 > solo_words ? top0 : solo_words;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < top; i += stride) {
        if (i < g.m && (flags & kInitLiveKey))
            s.live_key[i] = (flags & kInitLiveMark) ? ((uint64_t)g.w[i] << 32) | 1u
                            : s.key                 ? edge_key<true>(g, s, seed, (int)i)
                                                    : edge_key<false>(g, s, seed, (int)i);
        if (i < g.n) {
            s.best[0][i] = 0;
            s.done[i] = 0;
            if (flags & kInitHubs) {
                const int deg = g.v_off[i + 1] - g.v_off[i];
                if (deg >= s.hot_degree) hot += (unsigned long long)deg;
                if (deg > s.hub_threshold) {
                    const int np = (deg + kHubPiece - 1) / kHubPiece;
                    const int q0 = atomicAdd(s.piece_count, np);
                    for (int k = 0; k < np && q0 + k < s.piece_cap; ++k)
                        s.pieces[q0 + k] = make_int2((int)i, k);
                }
            }
        }
        if (i < words) bits[i] = 0;
        if (i < solo_words) s.solo[kSoloHeader + i] = 0;
    }
    if (flags & kInitHubs) {
        hot = block_sum_u64(hot, sum_tmp);
        if (threadIdx.x == 0 && hot) atomicAdd(&s.hot[blockIdx.x % kSub], hot);
    }
    if (flags & kInitWeightRange) reduce_weight_range(g, s);
}

// ---------------------------------------------------------------------------
// Validation (optional).  Edge side: e_off[0] = 0, offsets non-decreasing and
// at most kappa, e_off[m] = kappa, pins in [0, n), pins of an edge distinct.
// Vertex side (check_dual): the same for v_off / v_edges, and every
// vertex-side incidence (v, e) is found among e's pins at a position not
// claimed before (vbits, cleared by the host); with equal totals this makes
// the vertex side exactly the transpose.  Work: O(sum of |e|^2).
__global__ void __launch_bounds__(kBlock) k_validate(Graph g, State s, int check_dual) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kap = g.kappa;
    // Edge e's pins are e_pins[eoff(e) .. eoff(e + 1)).
    auto eoff = [&](int64_t e) -> int32_t { return g.pairs ? (int32_t)(2 * e) : g.e_off[e]; };
    if (tid0 == 0) {
        if (g.m > 0 && (eoff(0) != 0 || eoff(g.m) != kap)) atomicOr(s.err, 1);
        if (check_dual && (g.v_off[0] != 0 || g.v_off[g.n] != kap)) atomicOr(s.err, 2);
    }
    for (int64_t e = tid0; e < g.m; e += stride) {
        int32_t a = eoff(e), b = eoff(e + 1);
        if (b < a || a < 0 || b > kap) { atomicOr(s.err, 4); continue; }
        for (int32_t i = a; i < b; ++i) {
            int32_t p = g.e_pins[i];
            if (p < 0 || p >= g.n) { atomicOr(s.err, 8); break; }
            for (int32_t j = a; j < i; ++j)
                if (g.e_pins[j] == p) { atomicOr(s.err, 16); break; }
        }
    }
    if (!check_dual) return;
    for (int64_t v = tid0; v < g.n; v += stride) {
        int32_t a = g.v_off[v], b = g.v_off[v + 1];
        if (b < a || a < 0 || b > kap) { atomicOr(s.err, 32); continue; }
        for (int32_t i = a; i < b; ++i) {
            int32_t e = g.v_edges[i];
            if (e < 0 || e >= g.m) { atomicOr(s.err, 64); break; }
            int32_t ea = eoff(e), eb = eoff(e + 1);
            if (eb < ea || ea < 0 || eb > kap) { atomicOr(s.err, 64); break; }
            int32_t pos = -1;
            for (int32_t j = ea; j < eb && pos < 0; ++j)
                if (g.e_pins[j] == (int32_t)v) pos = j;
            if (pos < 0) { atomicOr(s.err, 128); break; }
            uint32_t bit = 1u << (pos & 31);
            if (atomicOr(&s.vbits[pos >> 5], bit) & bit) { atomicOr(s.err, 256); break; }
        }
    }
}

// ---------------------------------------------------------------------------
// Region helpers: number of live edges of workgroup b in round r, and item i.
__device__ __forceinline__ int region_count(const State &s, int m, int round, int b) {
    if (round == 0 && !s.explicit0) {
        const int64_t lo = (int64_t)b * s.region;
        const int64_t c = (int64_t)m - lo;
        return c <= 0 ? 0 : (c > s.region ? s.region : (int)c);
    }
    return s.cnt[round & 1][b];
}

__device__ __forceinline__ int region_item(const State &s, int round, int b, int i) {
    const int64_t at = (int64_t)b * s.region + i;
    return (round == 0 && !s.explicit0) ? (int)at : s.list[round & 1][at];
}

// Edge i of workgroup b's live list of round r, offset layout: id, pin offset
// and count, first pin (-1 if none), vertex base and key.  Round 0's list is
// the identity and reads the hypergraph.  Later lists read the records that
// the retire pass wrote beside the ids, at the same index, so one step
// replaces the gathers through the id.  rekey: the caller's round orders by a
// different seed than the list's round (per-round priorities), so the key is
// rebuilt from the weight.
struct EdgeRec {
    int e, base, len, pin0, vb;
    uint64_t key;
};

// key_round: the round whose key a rekeying caller needs.
template <bool kB>
__device__ __forceinline__ EdgeRec edge_rec(const Graph &g, const State &s, int round, int b,
                                            int i, uint32_t kseed, bool rekey, int key_round) {
    EdgeRec r;
    const int64_t at = (int64_t)b * s.region + i;
    if (round == 0 && !(kB && s.explicit0)) {
        r.e = (int)at;
        r.base = g.e_off[r.e];
        r.len = g.e_off[r.e + 1] - r.base;
        r.vb = kB ? g.vbase[r.e] : 0;
        r.key = rekey ? round_key<kB>(g, s, kseed, key_round, r.e) : edge_key<kB>(g, s, kseed, r.e);
        r.pin0 = r.len > 0 ? g.e_pins[r.base] + r.vb : -1;
    } else {
        const int k = round & 1;
        r.e = s.list[k][at];
        r.base = s.rec_a[k][at];
        r.len = s.rec_b[k][at];
        r.pin0 = s.rec_c[k][at];
        r.vb = kB ? s.rec_vb[k][at] : 0;
        r.key = rekey ? round_key<kB>(g, s, kseed, key_round, r.e) : s.rec_key[k][at];
    }
    return r;
}

// The same for the pair layout: id, both pins, key.
template <bool kB>
__device__ __forceinline__ void pair_rec(const Graph &g, const State &s, int round, int b, int i,
                                         uint32_t kseed, bool rekey, int &e, int2 &p,
                                         uint64_t &key) {
    const int64_t at = (int64_t)b * s.region + i;
    if (round == 0) {
        e = (int)at;
        p = pair_pins(g, e);
        key = rekey ? round_key<kB>(g, s, kseed, round + 1, e) : edge_key<kB>(g, s, kseed, e);
    } else {
        const int k = round & 1;
        e = s.list[k][at];
        p = make_int2(s.rec_a[k][at], s.rec_b[k][at]);
        key = rekey ? round_key<kB>(g, s, kseed, round + 1, e) : s.rec_key[k][at];
    }
}

// ---------------------------------------------------------------------------
// Edge-centric scatter of round 0 (Algorithm 1, per-vertex maximum by
// concurrent writes): every edge raises best[pin] to its key at each pin.
// The plain read first skips the atomic when the slot already holds a larger
// key; best only grows during the pass, so a stale read is merely cautious.
// With a hub table H (AUTO's round 0), hub pins are reduced in LDS and
// pushed once per workgroup at the end.
template <bool kPairs, bool kB>
__device__ __forceinline__ void scatter0_region(const Graph &g, const State &s, ChunkLds &L, int b,
                                                uint32_t kseed, HubTable *H = nullptr) {
    uint64_t *best = s.best[0];
    const int cnt = region_count(s, g.m, 0, b);
    if constexpr (kPairs) {
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            const int e = region_item(s, 0, b, i);
            scatter_pair(best, pair_pins(g, e), edge_key<kB>(g, s, kseed, e));
        }
        return;
    }
    for (int c0 = 0; c0 < cnt; c0 += kBlock) {
        const int i = c0 + threadIdx.x;
        int len = 0, base = 0;
        uint64_t key = 0;
        int vb = 0;
        if (i < cnt) {
            const int e = region_item(s, 0, b, i);
            base = g.e_off[e];
            len = g.e_off[e + 1] - base;
            key = edge_key<kB>(g, s, kseed, e);
            if constexpr (kB) vb = g.vbase[e];
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        L.vb[threadIdx.x] = vb;
        __syncthreads();
        if (H)
            scatter_chunk_hubs<kB>(L, g.e_pins, total, best, *H);
        else
            scatter_chunk<kB>(L, g.e_pins, total, best);
        __syncthreads();
    }
    if (H) {
        for (int i = threadIdx.x; i < kHubSlots; i += kBlock) {
            const int v = H->id[i];
            const uint64_t k = H->mx[i];
            if (v >= 0 && k && load_lower_bound(&best[v]) < k) atomic_max_u64(&best[v], k);
        }
    }
}

template <bool kPairs, bool kB>
__global__ void __launch_bounds__(kBlock) k_scatter0(Graph g, State s, uint32_t kseed) {
    __shared__ ChunkLds L;
    scatter0_region<kPairs, kB>(g, s, L, xcd_item(blockIdx.x, gridDim.x), kseed);
}

// ---------------------------------------------------------------------------
// Retire + compact (+ scatter) for round r >= 1.  Input: workgroup b's live
// edges of round r-1.  An edge survives iff it is non-empty and none of its
// pins is done; this removes the edges matched in round r-1 (all their pins
// are done) and every edge that touches them (Algorithm 2's OR-reduction over
// the pins of each edge).  Survivors are compacted, in order, into the
// workgroup's region of list[r & 1], each with its record (pin offset and
// count or the two pins, first pin, vertex base, round-r key) at the same
// index; the count goes to cnt[r & 1][b] and the round's counters.  rekey:
// round r orders by a different seed than round r-1, so keys are rebuilt
// from the weights instead of read from the input records.  Then, depending
// on the variant:
//   scatter = 1 (CRCW): each survivor raises best[r & 1][pin] at its pins.
//   scatter = 0 (CREW): non-survivors get live_key = 0, and the split hub
//                       vertices' best[r & 1] and vlen[r & 1] are cleared for
//                       the vertex pass.
// kPairs: graph layout; kScatter: the CRCW form (else CREW).  Each
// combination is its own kernel: a kernel holding every path runs the hot
// one slower.
// Binned form of the scatter (kBin, CRCW, one instance, offset layout): the
// first pass counts the survivors' non-hub pins per bin in LDS (bcnt) while
// hub pins are reduced in the hub table H, as in round 0's edge scatter.
// After the last chunk the workgroup reserves its run in every bin with one
// device atomic on the bin's cursor, pushes the hub maxima, and a second
// pass over its just-compacted survivors writes each non-hub pin's record
// into its run.  k_bin_max then reduces each bin.
constexpr uint32_t kBinOverflow = 0x80000000u;  // run position of a bin that overflowed

__device__ __forceinline__ void bin_count_chunk(const ChunkLds &L, const int32_t *e_pins,
                                                int total, HubTable &H, uint32_t *bcnt, int rb) {
    for (int t0 = threadIdx.x; t0 < total; t0 += kUnroll * kBlock) {
        int jj[kUnroll], pin[kUnroll];
        chunk_pins<false>(L, e_pins, total, t0, jj, pin);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (jj[u] < 0) continue;
            const int h = hub_find(H, pin[u]);
            if (h >= 0) {
                const unsigned long long k = L.key[jj[u]];
                if (H.mx[h] < k) atomicMax(&H.mx[h], k);
            } else {
                atomicAdd(&bcnt[pin[u] >> rb], 1u);
            }
        }
    }
}

__device__ __forceinline__ void bin_write_chunk(const ChunkLds &L, const int32_t *e_pins,
                                                int total, const HubTable &H, uint32_t *bpos,
                                                int rb, uint16_t *bin_v, uint64_t *bin_key) {
    const int mask = (1 << rb) - 1;
    for (int t0 = threadIdx.x; t0 < total; t0 += kUnroll * kBlock) {
        int jj[kUnroll], pin[kUnroll];
        chunk_pins<false>(L, e_pins, total, t0, jj, pin);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (jj[u] < 0 || hub_find(H, pin[u]) >= 0) continue;
            const uint32_t at = atomicAdd(&bpos[pin[u] >> rb], 1u);
            if (at < kBinOverflow) {
                bin_v[at] = (uint16_t)(pin[u] & mask);
                bin_key[at] = L.key[jj[u]];
            }
        }
    }
}

template <bool kPairs, bool kScatter, bool kB, bool kBin>
__device__ __forceinline__ void retire_body(const Graph &g, const State &s, int round,
                                            uint32_t kseed, int rekey, ChunkLds &L, HubTable *H,
                                            uint32_t *bcnt) {
    static_assert(!kBin || (kScatter && !kPairs && !kB), "bins: CRCW, one instance, offsets");
    constexpr bool scatter = kScatter;
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int cnt = region_count(s, g.m, round - 1, b);
    const int64_t out0 = (int64_t)b * s.region;  // the region's first list slot
    int32_t *out_list = s.list[round & 1] + out0;
    const int ko = round & 1;                     // records of the list written here
    uint64_t *best = s.best[round & 1];
    RoundStats *st_out = &s.stats[round % s.ring];

    if (!kScatter && b == 0) {
        const int np = min(*s.piece_count, s.piece_cap);
        for (int q = threadIdx.x; q < np; q += kBlock) {
            const int2 pc = s.pieces[q];
            if (pc.y == 0) {
                best[pc.x] = 0;
                if (s.vlen[0]) s.vlen[round & 1][pc.x] = 0;
            }
        }
    }
    if constexpr (kBin) {
        hub_table_build(*H, s);
        for (int j = threadIdx.x; j < s.bin_nb; j += kBlock) bcnt[j] = 0;
        __syncthreads();
    }
    int out_pos = 0;                 // survivors written so far (uniform)
    unsigned long long kap_acc = 0;  // their pins (thread 0's copy is the total)
    if constexpr (kPairs) {
        for (int c0 = 0; c0 < cnt; c0 += kBlock) {
            const int i = c0 + threadIdx.x;
            int e = -1, alive = 0;
            int2 p = make_int2(0, 0);
            uint64_t key = 0;
            if (i < cnt) {
                pair_rec<kB>(g, s, round - 1, b, i, kseed, rekey != 0, e, p, key);
                alive = (s.done[p.x] | s.done[p.y]) ? 0 : 1;
            }
            if (!scatter && e >= 0 && !alive) s.live_key[e] = 0;
            int n_alive;
            const int pos = block_exclusive_sum(alive, L.wave_tmp, &n_alive);
            if (alive) {
                const int64_t at = out0 + out_pos + pos;
                out_list[out_pos + pos] = e;
                s.rec_a[ko][at] = p.x;
                s.rec_b[ko][at] = p.y;
                s.rec_key[ko][at] = key;
                if (scatter) scatter_pair(best, p, key);
            }
            out_pos += n_alive;
        }
        kap_acc = 2ull * (unsigned long long)out_pos;
    }
    for (int c0 = 0; c0 < cnt && !kPairs; c0 += kBlock) {
        const int i = c0 + threadIdx.x;
        int e = -1, len = 0, base = 0, pin0 = -1;
        uint64_t key = 0;
        int vb = 0;
        if (i < cnt) {
            const EdgeRec r = edge_rec<kB>(g, s, round - 1, b, i, kseed, rekey != 0, round);
            e = r.e;
            base = r.base;
            len = r.len;
            pin0 = r.pin0;
            key = r.key;
            vb = r.vb;
        }
        // The first kUnroll pins one lane per edge: most retired edges are
        // found there, and most edges have no more pins.  The pins beyond
        // them, of the edges still undecided, are spread over all lanes of
        // the workgroup, kUnroll per lane and step, so that a long
        // surviving edge does not hold its wave for a chain of reads.
        bool dead = false;
        {
            int p[kUnroll];
            p[0] = len > 0 ? pin0 : -1;
#pragma unroll
            for (int u = 1; u < kUnroll; ++u) p[u] = u < len ? g.e_pins[base + u] + vb : -1;
            uint8_t dv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) dv[u] = p[u] >= 0 ? s.done[p[u]] : 0;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) dead |= dv[u] != 0;
        }
        {
            const int rest = (e >= 0 && !dead && len > kUnroll) ? len - kUnroll : 0;
            int total_r;
            const int st_r = block_exclusive_sum(rest, L.wave_tmp, &total_r);
            if (total_r > 0) {
                L.start[threadIdx.x] = st_r;
                L.base[threadIdx.x] = base + kUnroll;
                L.vb[threadIdx.x] = vb;
                L.flag[threadIdx.x] = 0;
                __syncthreads();
                for (int t0 = threadIdx.x; t0 < total_r; t0 += kUnroll * kBlock) {
                    int jj[kUnroll], pin[kUnroll];
                    chunk_pins<kB>(L, g.e_pins, total_r, t0, jj, pin);
                    uint8_t dv[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) dv[u] = jj[u] >= 0 ? s.done[pin[u]] : 0;
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (dv[u]) L.flag[jj[u]] = 1;
                }
                __syncthreads();
                dead = dead || L.flag[threadIdx.x];
                __syncthreads();
            }
        }
        const int alive = (e >= 0 && len > 0 && !dead) ? 1 : 0;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        L.vb[threadIdx.x] = vb;
        if (!scatter && e >= 0 && !alive) s.live_key[e] = 0;
        int n_alive;
        int pos = block_exclusive_sum(alive, L.wave_tmp, &n_alive);
        if (alive) {
            const int64_t at = out0 + out_pos + pos;
            out_list[out_pos + pos] = e;
            s.rec_a[ko][at] = base;
            s.rec_b[ko][at] = len;
            s.rec_c[ko][at] = pin0;
            if constexpr (kB) s.rec_vb[ko][at] = vb;
            s.rec_key[ko][at] = key;
        }
        out_pos += n_alive;
        int total2;
        int st2 = block_exclusive_sum(alive ? len : 0, L.wave_tmp, &total2);
        kap_acc += (unsigned long long)total2;
        if (scatter) {
            L.start[threadIdx.x] = st2;
            __syncthreads();
            if constexpr (kBin)
                bin_count_chunk(L, g.e_pins, total2, *H, bcnt, s.bin_rb);
            else
                scatter_chunk<kB>(L, g.e_pins, total2, best);
        }
        __syncthreads();
    }
    if constexpr (kBin) {
        // Runs: bin j's records of this workgroup go to bpos[j] onwards.
        uint32_t *bpos = bcnt + s.bin_nb;
        const int rb = s.bin_rb;
        for (int j = threadIdx.x; j < s.bin_nb; j += kBlock) {
            const uint32_t c = bcnt[j];
            uint32_t p = 0;
            if (c) {
                const int64_t v0 = (int64_t)j << rb;
                const int lo = g.v_off[v0];
                const int hi = g.v_off[min(v0 + ((int64_t)1 << rb), (int64_t)g.n)];
                const uint32_t got = atomicAdd(&s.bin_cursor[j], c);
                if (lo < 0 || hi > g.kappa || (int64_t)lo + got + c > (int64_t)hi) {
                    p = kBinOverflow;
                    atomicAdd(&st_out->bin_overflow, 1ull);
                } else {
                    p = (uint32_t)lo + got;
                }
            }
            bpos[j] = p;
        }
        for (int i = threadIdx.x; i < kHubSlots; i += kBlock) {
            const int v = H->id[i];
            const uint64_t k = H->mx[i];
            if (v >= 0 && k && load_lower_bound(&best[v]) < k) atomic_max_u64(&best[v], k);
        }
        __syncthreads();
        // Second pass over the survivors this workgroup compacted above (its
        // own writes, visible after the barrier).
        for (int c0 = 0; c0 < out_pos; c0 += kBlock) {
            const int i = c0 + threadIdx.x;
            int len = 0, base = 0;
            uint64_t key = 0;
            if (i < out_pos) {
                const int64_t at = out0 + i;
                base = s.rec_a[ko][at];
                len = s.rec_b[ko][at];
                key = s.rec_key[ko][at];
            }
            int total;
            const int st = block_exclusive_sum(len, L.wave_tmp, &total);
            L.start[threadIdx.x] = st;
            L.base[threadIdx.x] = base;
            L.key[threadIdx.x] = key;
            __syncthreads();
            bin_write_chunk(L, g.e_pins, total, *H, bpos, rb, s.bin_v, s.bin_key);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        s.cnt[round & 1][b] = out_pos;
        if (out_pos > 0) {
            atomicAdd(&st_out->live[b % kSub], (unsigned long long)out_pos);
            atomicAdd(&st_out->kappa[b % kSub], kap_acc);
        }
    }
}

template <bool kPairs, bool kScatter, bool kB>
__global__ void __launch_bounds__(kBlock) k_retire(Graph g, State s, int round, uint32_t kseed,
                                                   int rekey) {
    __shared__ ChunkLds L;
    retire_body<kPairs, kScatter, kB, false>(g, s, round, kseed, rekey, L, nullptr, nullptr);
}

__device__ __forceinline__ bool max0_edge_form(const Graph &g, const State &s);

// Whether the binned form runs: always with an explicit bin size; with the
// automatic one only where round 0 took the vertex form, i.e. most pins lie
// on vertices below the hot degree.  There a vertex sees few records per
// round, so nearly every filtered read is followed by its atomic; on skewed
// degrees the filter stops most of them and the atomic scatter is faster.
__device__ __forceinline__ bool bins_run(const Graph &g, const State &s) {
    return !s.bin_auto || !max0_edge_form(g, s);
}

// The binned form; dynamic LDS: bin counts, then run positions (2 bin_nb
// words).  Where bins_run says no, the atomic scatter instead.
__global__ void __launch_bounds__(kBlock) k_retire_bin(Graph g, State s, int round,
                                                       uint32_t kseed, int rekey) {
    __shared__ ChunkLds L;
    __shared__ HubTable H;
    extern __shared__ uint32_t bcnt[];
    if (bins_run(g, s))
        retire_body<false, true, false, true>(g, s, round, kseed, rekey, L, &H, bcnt);
    else
        retire_body<false, true, false, false>(g, s, round, kseed, rekey, L, nullptr, nullptr);
}

// Reduces bin j (workgroup j): the maximum key of each of its vertices over
// the records the retire pass wrote, in an LDS tile of 2^bin_rb keys, then
// raised into best[round & 1] where nonzero (the test cleared the others, as
// for the atomic form; hub vertices got theirs from the retire pass).  Resets
// the bin's cursor for the next round.
__global__ void __launch_bounds__(kBinThreads) k_bin_max(Graph g, State s, int round) {
    extern __shared__ unsigned long long tile[];
    if (!bins_run(g, s)) return;  // the retire pass scattered by atomics
    const int j = blockIdx.x;
    const int rb = s.bin_rb;
    const int64_t v0 = (int64_t)j << rb;
    const int64_t v1 = min(v0 + ((int64_t)1 << rb), (int64_t)g.n);
    const int lo = max(g.v_off[v0], 0);
    const int hi = (int)min((int64_t)g.v_off[v1], g.kappa);
    const int64_t c = min((int64_t)s.bin_cursor[j], (int64_t)hi - lo);  // < 0: nothing
    const int nv = (int)(v1 - v0);
    for (int t = threadIdx.x; t < nv; t += kBinThreads) tile[t] = 0;
    __syncthreads();
    const uint16_t *bv = s.bin_v + lo;
    const uint64_t *bk = s.bin_key + lo;
    constexpr int64_t step = (int64_t)kUnroll * kBinThreads;
    for (int64_t i0 = threadIdx.x; i0 < c; i0 += step) {
        uint16_t v[kUnroll];
        uint64_t k[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBinThreads;
            v[u] = i < c ? bv[i] : 0;
            k[u] = i < c ? bk[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (k[u] && v[u] < nv) atomicMax(&tile[v[u]], (unsigned long long)k[u]);
    }
    __syncthreads();
    // Only this workgroup writes the bin's entries during the kernel; an entry
    // may already hold a hub maximum pushed by the retire pass (a workgroup
    // whose table holds a hub that another workgroup's full table left out
    // sends it to the bins instead), so the larger of the two stays.
    uint64_t *best = s.best[round & 1];
    for (int t = threadIdx.x; t < nv; t += kBinThreads) {
        const uint64_t x = tile[t];
        if (x && x > best[v0 + t]) best[v0 + t] = x;
    }
    if (threadIdx.x == 0) s.bin_cursor[j] = 0;
}

// ---------------------------------------------------------------------------
// Vertex-centric maximum of round r (Algorithm 2, segmented MAX over each
// vertex's incidence list).  Chunks of kBlock consecutive vertices: done
// vertices and split hubs contribute no incidences; the chunk's incidences
// are flattened over the lanes, each wave reduces runs of equal vertex with a
// segmented max-scan in registers, and one LDS atomic per run and wave
// combines the runs.  Hubs (degree > hub threshold) are cut into pieces of
// kHubPiece incidences, each reduced by one workgroup and combined with one
// global atomic max (their best was cleared by init or the retire pass).
// Round 0 has no retired edge yet: keys are rebuilt from the weights
// (w << 32 | H(seed, e)), gathering 4 bytes per incidence instead of 8;
// later rounds gather live_key (0 once the edge left the live set).
//
// Work-optimal lists (Section 5.2.3, the rebuilt incidence arrays): from
// round 1 on the pass also writes each open vertex's live incident edges to
// the front of its segment of vedges[r & 1] (same offsets as v_off, any
// order, global edge ids) with the count in vlen[r & 1], and round r + 1
// reads those lists instead of the full ones.  A round thus reads only the
// incidences that were live one round earlier instead of every open vertex's
// whole list.  Round 1 reads the caller's lists.  Non-hub positions come from
// an LDS counter per vertex; a hub's from one global atomic per wave on its
// vlen entry (cleared by the retire pass).
// The weight range k_init left in kSub slots: smallest weight, and whether
// every weight equals it (false when there are no edges).
__device__ __forceinline__ void weight_range(const State &s, uint32_t *wlo, bool *uniform) {
    __shared__ uint32_t lo, hi;
    if (threadIdx.x < kWave) {
        uint32_t a = threadIdx.x < kSub ? s.wrange[2 * threadIdx.x] : 0xFFFFFFFFu;
        uint32_t c = threadIdx.x < kSub ? s.wrange[2 * threadIdx.x + 1] : 0;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const uint32_t a2 = __shfl_xor(a, o, kWave), c2 = __shfl_xor(c, o, kWave);
            a = a2 < a ? a2 : a;
            c = c2 > c ? c2 : c;
        }
        if (threadIdx.x == 0) {
            lo = a;
            hi = c;
        }
    }
    __syncthreads();
    *wlo = lo;
    *uniform = lo == hi;
}

// Key of incident edge e in the vertex pass of round r, and whether e is
// live.  uniform_w: every weight equals wlo (one instance, round 0), so the
// key needs no gather.  From round 1 on live_key says whether e is live; it
// holds the key itself, or with rekey (priorities redrawn every round) a
// liveness mark with the weight, and the key is rebuilt for the round.  A
// live edge whose key is 0 is kept in the lists: with rekey its key changes.
template <bool kB>
__device__ __forceinline__ uint64_t vertex_key(const Graph &g, const State &s, int round,
                                               uint32_t seed, int e, bool uniform_w,
                                               uint32_t wlo, bool rekey, bool *live) {
    *live = true;
    if (!kB && round == 0 && uniform_w)
        return ((uint64_t)wlo << 32) | priority_hash(seed, (uint32_t)e);
    if (round == 0) return edge_key<kB>(g, s, seed, e);
    const uint64_t lk = s.live_key[e];
    *live = lk != 0;
    return (rekey && lk) ? round_key<kB>(g, s, seed, round, e) : lk;
}

// kCompact: rounds >= 1 (list compaction); round 0 instantiates without it.
template <bool kCompact, bool kB>
__device__ __forceinline__ void vertex_max_body(const Graph &g, const State &s, ChunkLds &L,
                                                int round, uint32_t seed, bool rekey) {
    uint64_t *best = s.best[round & 1];
    const int lane = threadIdx.x & (kWave - 1);
    const int hub_threshold = s.hub_threshold;
    // Round 0 of one instance: k_init left the weight range (all equal:
    // keys without a gather).  Other rounds gather stored keys.
    uint32_t wlo = 0;
    bool uniform_w = false;
    if (!kB && round == 0) weight_range(s, &wlo, &uniform_w);
    constexpr bool compact = kCompact;
    // Lists read this round: the caller's (local ids in a batch, full degree)
    // up to round 1, then the ones compacted by the previous round.
    const bool caller_lists = !kCompact || round <= 1;
    const int32_t *src = caller_lists ? g.v_edges : s.vedges[(round - 1) & 1];
    const int32_t *src_len = caller_lists ? nullptr : s.vlen[(round - 1) & 1];
    int32_t *dst = compact ? s.vedges[round & 1] : nullptr;
    int32_t *dst_len = compact ? s.vlen[round & 1] : nullptr;

    const int n_pieces = min(*s.piece_count, s.piece_cap);
    for (int q = blockIdx.x; q < n_pieces; q += gridDim.x) {
        const int2 pc = s.pieces[q];
        const int v = pc.x;
        if (s.done[v]) continue;
        const int vo = g.v_off[v];
        const int len = src_len ? src_len[v] : g.v_off[v + 1] - vo;
        const int p0 = pc.y * kHubPiece;
        if (p0 >= len) continue;
        const int p1 = min(len, p0 + kHubPiece);
        const int eb = (kB && caller_lists) ? g.ebase[v] : 0;
        uint64_t mx = 0;
        for (int i0 = p0; i0 < p1; i0 += kBlock) {  // uniform trip count (ballot below)
            const int i = i0 + threadIdx.x;
            int e = -1;
            uint64_t k = 0;
            bool live = false;
            if (i < p1) {
                e = src[vo + i] + eb;
                k = vertex_key<kB>(g, s, round, seed, e, uniform_w, wlo, rekey, &live);
            }
            mx = k > mx ? k : mx;
            if constexpr (compact) {
                const unsigned long long mask = __ballot(live);
                const int cnt = __popcll(mask);
                int at = 0;
                if (lane == 0 && cnt) at = atomicAdd(&dst_len[v], cnt);
                at = __shfl(at, 0, kWave);
                if (live) dst[vo + at + __popcll(mask & ((1ull << lane) - 1))] = e;
            }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            uint64_t y = __shfl_xor(mx, o, kWave);
            mx = y > mx ? y : mx;
        }
        if (lane == 0 && mx) atomic_max_u64(&best[v], mx);
    }

    // The grid sweeps the vertices in steps of gridDim.x chunks (all
    // workgroups work on neighbouring vertices at a time); within a step each
    // XCD takes one contiguous share (xcd_item).
    for (int64_t c0 = (int64_t)xcd_item(blockIdx.x, gridDim.x) * kBlock; c0 < g.n;
         c0 += (int64_t)gridDim.x * kBlock) {
        const int v = (int)c0 + threadIdx.x;
        int len = 0, base = 0, eb = 0;
        bool own = false;
        if (v < g.n && !s.done[v]) {
            base = g.v_off[v];
            own = g.v_off[v + 1] - base <= hub_threshold;
            if (own) len = src_len ? src_len[v] : g.v_off[v + 1] - base;
            if (kB && caller_lists) eb = g.ebase[v];
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = 0;
        L.vb[threadIdx.x] = eb;
        L.flag[threadIdx.x] = 0;  // live incidences kept so far
        __syncthreads();
        for (int t0 = 0; t0 < total; t0 += kBlock) {
            const int t = t0 + threadIdx.x;
            int j = -1;
            uint64_t k = 0;
            if (t < total) {
                j = find_item(L.start, t);
                const int e = src[L.base[j] + (t - L.start[j])] + (kB ? L.vb[j] : 0);
                bool live;
                k = vertex_key<kB>(g, s, round, seed, e, uniform_w, wlo, rekey, &live);
                if constexpr (compact) {
                    if (live) dst[L.base[j] + atomicAdd(&L.flag[j], 1)] = e;
                }
            }
            // segmented inclusive max-scan over the wave, segments = equal j
            k = wave_segmented_max(k, j);
            const bool last = next_lane_j(j) != j;  // lane 63 reads -2
            if (j >= 0 && last && k) atomicMax((unsigned long long *)&L.key[j], (unsigned long long)k);
        }
        __syncthreads();
        if (own) {
            best[v] = L.key[threadIdx.x];
            if constexpr (compact) dst_len[v] = L.flag[threadIdx.x];
        }
        __syncthreads();
    }
}

// seed: the round's priority seed (one instance); rekey: priorities are
// redrawn every round, so keys are rebuilt instead of read from live_key.
template <bool kB>
__global__ void __launch_bounds__(kBlock) k_vertex_max(Graph g, State s, int round, uint32_t seed,
                                                       int rekey) {
    __shared__ ChunkLds L;
    if (round == 0)
        vertex_max_body<false, kB>(g, s, L, round, seed, false);
    else
        vertex_max_body<true, kB>(g, s, L, round, seed, rekey != 0);
}

// Round-0 maximum when the library chooses the form (AUTO).  The edge-centric
// scatter pays one L2-cached read per incidence and an atomic only where the
// key raises the maximum, so it is fastest when most incidences fall on a few
// hot vertices whose entries stay in L2; the vertex-centric pass gathers one
// weight per incidence with no atomics, which is faster when incidences are
// spread evenly.  k_init counted the incidences of vertices of degree >=
// the hot degree; the edge form is taken when they are at least half of all.
// The edge form reduces the hubs' pins in each workgroup's hub table.
// Two kernels, each running only when the form is its own: the edge form
// with its hub table and the vertex form are compiled separately (one kernel
// holding both ran the vertex form 7% slower).  Both read the form from the
// degree profile on the device, so the host needs no synchronisation.
__device__ __forceinline__ bool max0_edge_form(const Graph &g, const State &s) {
    __shared__ int edge_form;
    if (threadIdx.x < kWave) {
        unsigned long long hot = s.hot[threadIdx.x];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) hot += __shfl_xor(hot, o, kWave);
        if (threadIdx.x == 0) edge_form = 2 * hot >= (unsigned long long)g.kappa;
    }
    __syncthreads();
    return edge_form != 0;
}

template <bool kPairs, bool kB>
__global__ void __launch_bounds__(kBlock) k_max0_edge(Graph g, State s, uint32_t seed) {
    __shared__ ChunkLds L;
    __shared__ HubTable H;
    const bool edge_form = max0_edge_form(g, s);
    if (blockIdx.x == 0 && threadIdx.x == 0) s.stats[0].form = edge_form ? 1 : 2;
    if (!edge_form) {
        // The vertex form follows: its keys need no weight gather when all
        // weights are equal (one instance), which the range shows.
        if constexpr (!kB) reduce_weight_range(g, s);
        return;
    }
    hub_table_build(H, s);
    scatter0_region<kPairs, kB>(g, s, L, xcd_item(blockIdx.x, gridDim.x), seed, &H);
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_max0_vertex(Graph g, State s, uint32_t seed) {
    __shared__ ChunkLds L;
    if (max0_edge_form(g, s)) return;
    vertex_max_body<false, kB>(g, s, L, 0, seed, false);
}

// ---------------------------------------------------------------------------
// Local-max test of round r (Algorithm 1 third phase; Algorithm 2 P_e = |e|):
// a live edge is matched iff best[v] == key(e) at every pin v.  Matched edges
// set their bitmap bit and mark their pins done (exclusive: a vertex has one
// maximum edge).
// kClear says how the next round's buffer best[(r+1) & 1] is zeroed for the
// next scatter (the next round's survivors are a subset of this round's
// live edges, so zero at every pin this pass reads is enough):
//   kClearNone  the next round is vertex-centric (it writes every entry)
//   kClearAll   one streaming pass over all n entries, for rounds with many
//               pins (a full sequential clear is cheaper than as many
//               scattered stores); the test itself stops at the first pin
//               where the edge is not the maximum
//   kClearPins  a store at every pin of every live edge, all pins visited
// The host picks the form from its latest count of live pins; any form is
// correct.  Workgroup 0 also clears the counters of round r+1.
constexpr int kTestEdges = 2;  // edges per lane and step of the early-exit test

// kPairs: graph layout (instantiated separately; g.pairs equals it).
template <bool kPairs, int kClear, bool kB>
__global__ void __launch_bounds__(kBlock) k_test(Graph g, State s, int round, uint32_t *bits,
                                                 uint32_t kseed) {
    __shared__ ChunkLds L;
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int cnt = region_count(s, g.m, round, b);
    const uint64_t *best = s.best[round & 1];
    uint64_t *next = s.best[(round + 1) & 1];
    RoundStats *st_cur = &s.stats[round % s.ring];
    if (b == 0) {
        unsigned long long *z = (unsigned long long *)&s.stats[(round + 1) % s.ring];
        for (int i = threadIdx.x; i < (int)(sizeof(RoundStats) / 8); i += kBlock) z[i] = 0;
    }
    if constexpr (kClear == kClearAll) {
        const int64_t stride = (int64_t)gridDim.x * kBlock;
        for (int64_t v = (int64_t)b * kBlock + threadIdx.x; v < g.n; v += stride) next[v] = 0;
    }
    if (cnt == 0) return;  // an empty region (most of them in late rounds): no counters
    constexpr bool clear_pins = kClear == kClearPins;
    unsigned long long nm = 0, wm = 0, pm = 0;  // per-thread partial counters
    if constexpr (kPairs) {
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            int e;
            int2 p;
            uint64_t key;
            pair_rec<kB>(g, s, round, b, i, kseed, false, e, p, key);
            const uint64_t b0 = best[p.x], b1 = best[p.y];
            if constexpr (clear_pins) {
                next[p.x] = 0;
                next[p.y] = 0;
            }
            if (b0 == key && b1 == key) {
                const int bit = kB ? e + g.bitoff[e] : e;
                atomicOr(&bits[bit >> 5], 1u << (bit & 31));
                nm += 1;
                wm += key >> 32;
                pm += 2;
                s.done[p.x] = 1;
                s.done[p.y] = 1;
            }
        }
    }
    // A matched edge sets its bit and marks its pins (no other live edge
    // shares a pin with it in this round).
    auto record = [&](int e, int base, int len, int vb, uint64_t key) {
        const int bit = kB ? e + g.bitoff[e] : e;
        atomicOr(&bits[bit >> 5], 1u << (bit & 31));
        nm += 1;
        wm += key >> 32;
        pm += (unsigned long long)len;
        for (int k = 0; k < len; ++k) s.done[g.e_pins[base + k] + vb] = 1;
    };
    if (!kPairs && !clear_pins) {
        // One lane per edge, stopping at the first pin where the edge is not
        // the maximum: almost every edge fails at its first pin.  A lane
        // takes kTestEdges edges per step with their loads issued together,
        // so their dependent chains (id, offsets, pin, maximum) overlap.
        for (int c0 = 0; c0 < cnt; c0 += kTestEdges * kBlock) {
            int e[kTestEdges], len[kTestEdges], base[kTestEdges], vb[kTestEdges], pin0[kTestEdges];
            uint64_t key[kTestEdges];
            bool ok[kTestEdges];
#pragma unroll
            for (int u = 0; u < kTestEdges; ++u) {
                const int i = c0 + u * kBlock + threadIdx.x;
                e[u] = -1;
                len[u] = base[u] = vb[u] = 0;
                pin0[u] = -1;
                key[u] = 0;
                if (i < cnt) {
                    const EdgeRec r = edge_rec<kB>(g, s, round, b, i, kseed, false, round);
                    e[u] = r.e;
                    base[u] = r.base;
                    len[u] = r.len;
                    pin0[u] = r.pin0;
                    key[u] = r.key;
                    vb[u] = r.vb;
                }
            }
#pragma unroll
            for (int u = 0; u < kTestEdges; ++u)
                ok[u] = e[u] >= 0 && (len[u] == 0 || best[pin0[u]] == key[u]);
#pragma unroll
            for (int u = 0; u < kTestEdges; ++u) {
                // the rest of the pins, kUnroll at a time, while still the maximum
                for (int k0 = 1; k0 < len[u] && ok[u]; k0 += kUnroll) {
                    int p[kUnroll];
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q)
                        p[q] = k0 + q < len[u] ? g.e_pins[base[u] + k0 + q] + vb[u] : -1;
                    uint64_t bv[kUnroll];
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q) bv[q] = p[q] >= 0 ? best[p[q]] : key[u];
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q) ok[u] = ok[u] && bv[q] == key[u];
                }
                if (ok[u]) record(e[u], base[u], len[u], vb[u], key[u]);
            }
        }
    }
    for (int c0 = 0; c0 < cnt && !kPairs && clear_pins; c0 += kBlock) {
        // Every pin is visited (its next-round entry is cleared), spread over
        // the lanes.
        const int i = c0 + threadIdx.x;
        int e = -1, len = 0, base = 0;
        uint64_t key = 0;
        int vb = 0;
        if (i < cnt) {
            const EdgeRec r = edge_rec<kB>(g, s, round, b, i, kseed, false, round);
            e = r.e;
            base = r.base;
            len = r.len;
            key = r.key;
            vb = r.vb;
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        L.flag[threadIdx.x] = 0;
        L.vb[threadIdx.x] = vb;
        __syncthreads();
        for (int t0 = threadIdx.x; t0 < total; t0 += kUnroll * kBlock) {
            int j[kUnroll], pin[kUnroll];
            chunk_pins<kB>(L, g.e_pins, total, t0, j, pin);
            uint64_t bv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) bv[u] = j[u] >= 0 ? best[pin[u]] : 0;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (j[u] < 0) continue;
                if (bv[u] != L.key[j[u]]) L.flag[j[u]] = 1;
                next[pin[u]] = 0;
            }
        }
        __syncthreads();
        const bool matched = e >= 0 && !L.flag[threadIdx.x];
        __syncthreads();
        if (matched) record(e, base, len, vb, key);
    }
    nm = block_sum_u64(nm, L.sum_tmp);
    wm = block_sum_u64(wm, L.sum_tmp);
    pm = block_sum_u64(pm, L.sum_tmp);
    if (threadIdx.x == 0 && nm) {
        atomicAdd(&st_cur->matched[b % kSub], nm);
        atomicAdd(&st_cur->weight[b % kSub], wm);
        atomicAdd(&st_cur->mpins[b % kSub], pm);
    }
}

// Batch setup: global pin and incidence offsets, per-edge vertex base and
// bitmap offset, per-vertex edge base, and keys w << 32 | H(seed_i, local id)
// with each instance's own seed.  Each instance's bitmap starts at bit
// 32 * word_base[i].  Work is balanced over items, not instances (instance
// sizes span orders of magnitude): workgroup b takes the b-th contiguous
// range of edges, then of vertices; one binary search finds the instance at
// the range's start, and each lane moves forward over instance boundaries as
// its item advances through the range.

// Largest i in [0, count) with base[i] <= x: the instance holding item x
// (base non-decreasing, base[0] = 0, base[count] > x; empty instances are
// skipped because a later instance with the same base is larger).
__device__ __forceinline__ int instance_of(const int64_t *base, int count, int64_t x) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// This workgroup's range [lo, hi) of `total` items, a multiple of kBlock long.
__device__ __forceinline__ void block_range(int64_t total, int64_t *lo, int64_t *hi) {
    const int64_t per =
        ((total + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    *lo = (int64_t)blockIdx.x * per;
    *hi = *lo + per < total ? *lo + per : total;
}

__global__ void __launch_bounds__(kBlock) k_batch_setup(Graph g, BatchIn b, State s) {
    __shared__ int first;
    int64_t lo, hi;
    block_range(g.m, &lo, &hi);
    if (lo < hi) {
        if (threadIdx.x == 0) first = instance_of(b.e_base, b.count, lo);
        __syncthreads();
        int i = first;
        for (int64_t e = lo + threadIdx.x; e < hi; e += kBlock) {
            while (i + 1 < b.count && b.e_base[i + 1] <= e) ++i;
            const int64_t eb = b.e_base[i], el = e - eb;
            b.goff[e] = (int32_t)(b.pin_base[i] + b.e_off[eb + i + el]);
            b.vbase[e] = (int32_t)b.v_base[i];
            b.bitoff[e] = (int32_t)(32 * b.word_base[i] - eb);
            const uint32_t sd = b.seeds[i];
            s.key[e] = ((uint64_t)g.w[e] << 32) |
                       priority_hash(b.reseed ? round_seed(sd, 0) : sd, (uint32_t)el);
            if (b.reseed) s.eseed[e] = ((uint64_t)sd << 32) | (uint32_t)el;
        }
        __syncthreads();  // `first` is reused below
    }
    if (b.gvoff) {
        block_range(g.n, &lo, &hi);
        if (lo < hi) {
            if (threadIdx.x == 0) first = instance_of(b.v_base, b.count, lo);
            __syncthreads();
            int i = first;
            for (int64_t v = lo + threadIdx.x; v < hi; v += kBlock) {
                while (i + 1 < b.count && b.v_base[i + 1] <= v) ++i;
                const int64_t vb = b.v_base[i];
                b.gvoff[v] = (int32_t)(b.pin_base[i] + b.v_off[vb + i + (v - vb)]);
                b.ebase[v] = (int32_t)b.e_base[i];
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.goff[g.m] = (int32_t)b.pin_base[b.count];
        if (b.gvoff) b.gvoff[g.n] = (int32_t)b.pin_base[b.count];
    }
}

// ---------------------------------------------------------------------------
// Solo part of a batch: one workgroup matches one small instance from its
// first round to its last, with only workgroup barriers between the phases
// of a round, so a small instance pays no kernel launch and no grid-wide
// pass per round and ends its own rounds when its own live list is empty.
// Workgroups take instances from a counter.  Round 0 starts with every edge
// raising best at its pins; then each round:
//   test    a live edge whose key equals best at every pin is matched: its
//           bit is set and its pins are marked done (Algorithm 2, P_e = |e|)
//   clear   best of the instance is zeroed
//   retire  every other live edge with a done pin leaves the live list
//           (soft delete); the survivors are compacted, in order, into the
//           other list and raise best at their pins with their key of the
//           next round (Algorithm 1's concurrent maximum)
// Vertex ids inside an instance are its local ids, so best and done are
// indexed by them directly: in LDS when the instance has at most lds_verts
// vertices (kLds), else in the workspace's arrays at its vertex range.  The
// lists are edge-local ids in list[0] / list[1] at the instance's edge range
// (free until k_live0_place builds the round kernels' lists).
constexpr int kSoloWaves = kSoloThreads / kWave;

__device__ __forceinline__ int solo_exclusive_sum(int v, int *wave_tmp, int *total) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) wave_tmp[wid] = incl;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kSoloWaves; ++i) {
        const int x = wave_tmp[i];
        off += (i < wid) ? x : 0;
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return off + incl - v;
}

__device__ __forceinline__ unsigned long long solo_sum(unsigned long long v,
                                                       unsigned long long *tmp) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) tmp[wid] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int i = 0; i < kSoloWaves; ++i) t += tmp[i];
    __syncthreads();
    return t;
}

// Key of (global) edge gl in round r of a batch.
__device__ __forceinline__ uint64_t solo_key(const Graph &g, const State &s, int gl, int r,
                                             bool rekey) {
    return rekey ? round_key<true>(g, s, 0, r, gl) : s.key[gl];
}

// Shared memory of one chunk of kSoloThreads live edges (flattened pin loops).
struct SoloChunk {
    int start[kSoloThreads];   // exclusive scan of the pins each edge contributes
    int base[kSoloThreads];    // offset of those pins in e_pins
    uint64_t key[kSoloThreads];
    int flag[kSoloThreads];
    int wave_tmp[kSoloWaves];
    unsigned long long sum_tmp[kSoloWaves];
    int inst;
};
static_assert(sizeof(SoloChunk) + 256 <= kSoloStaticLds, "k_solo's shared variables");

// Largest j in [0, kSoloThreads) with start[j] <= t.
__device__ __forceinline__ int solo_find(const int *start, int t) {
    int j = 0;
#pragma unroll
    for (int step = kSoloThreads / 2; step > 0; step >>= 1)
        if (start[j + step] <= t) j += step;
    return j;
}

// The kUnroll incidences t0, t0 + kSoloThreads, ... of a chunk: edge slot
// j (-1 past the end) and pin, all loads issued before any is used.
__device__ __forceinline__ void solo_pins(const SoloChunk &C, const int32_t *e_pins, int total,
                                          int t0, int (&j)[kUnroll], int (&pin)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int t = t0 + u * kSoloThreads;
        j[u] = t < total ? solo_find(C.start, t) : -1;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
        pin[u] = j[u] >= 0 ? e_pins[C.base[j[u]] + (t0 + u * kSoloThreads - C.start[j[u]])] : 0;
}

__device__ __forceinline__ bool bit_is_set(const uint32_t *bits, int v) {
    return (bits[v >> 5] >> (v & 31)) & 1u;
}

// One instance, every round, in this workgroup.  The instance's vertex ids
// are its local ids.  done is a bitmask in LDS; best is kept in LDS in tiles
// of `tile` vertices.  With one tile (most instances) a round is: test (first
// pin per lane, the rest of the undecided edges spread over the workgroup),
// clear, and retire fused with the next round's maximum.  With several tiles
// a round first forms the maximum and tests it tile by tile, each pass
// streaming the live pins and keeping those inside the tile, the failed
// tests collected in a flag per live edge (in the workspace); then matched
// edges are marked and the retire pass compacts the survivors.
__device__ __forceinline__ void solo_run(const Graph &g, const State &s, const SoloArgs &a,
                                         uint32_t *bits, bool rekey, int inst,
                                         unsigned char *lds, SoloChunk &C) {
    const int tid = threadIdx.x;
    const int64_t v0 = a.v_base[inst], e0 = a.e_base[inst];
    const int nv = (int)(a.v_base[inst + 1] - v0);
    const int ne = (int)(a.e_base[inst + 1] - e0);
    const int64_t bit0 = 32 * a.word_base[inst];
    const int32_t *e_pins = g.e_pins;
    const int dwords = (nv + 31) >> 5;
    uint32_t *done = reinterpret_cast<uint32_t *>(lds);
    const int dbytes = ((4 * dwords + 255) / 256) * 256;
    uint64_t *best = reinterpret_cast<uint64_t *>(lds + dbytes);
    const int tile = (a.lds_bytes - dbytes) / 8;
    const int tiles = (nv + tile - 1) / tile;
    const bool one = tiles <= 1;
    int32_t *const list0 = s.list[0] + e0, *const list1 = s.list[1] + e0;
    int32_t *const fail = s.rec_a[0] + e0;  // per live position (several tiles)
    for (int w = tid; w < dwords; w += kSoloThreads) done[w] = 0;

    // Raises best[pin - lo] to each chunk edge's key at its pins in [lo, hi).
    auto scatter = [&](int total, int lo, int hi) {
        for (int t0 = tid; t0 < total; t0 += kUnroll * kSoloThreads) {
            int j[kUnroll], pin[kUnroll];
            solo_pins(C, e_pins, total, t0, j, pin);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (j[u] >= 0 && pin[u] >= lo && pin[u] < hi)
                    atomicMax((unsigned long long *)&best[pin[u] - lo],
                              (unsigned long long)C.key[j[u]]);
        }
    };
    // Chunk of live edges c0.. of list `in` (identity in round 0): loads one
    // edge per lane and scans `contrib` of the pins into C (start, base).
    auto edge_of = [&](const int32_t *in, int r, int j, int &e, int &base, int &len) {
        e = r == 0 ? j : in[j];
        const int gl = (int)e0 + e;
        base = g.e_off[gl];
        len = g.e_off[gl + 1] - base;
    };
    // Sets the bit, counts and marks the pins of matched edge e.
    unsigned long long nm = 0, wm = 0, pm = 0;
    auto record = [&](int e, int base, int len, uint64_t key) {
        const int64_t bit = bit0 + e;
        atomicOr(&bits[bit >> 5], 1u << (bit & 31));
        nm += 1;
        wm += key >> 32;
        pm += (unsigned long long)len;
        for (int k0 = 0; k0 < len; k0 += kUnroll) {
            int p[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) p[u] = k0 + u < len ? e_pins[base + k0 + u] : -1;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (p[u] >= 0) atomicOr(&done[p[u] >> 5], 1u << (p[u] & 31));
        }
    };
    // The maximum of round r over the tile [lo, hi) of the live edges.
    auto max_pass = [&](const int32_t *in, int r, int E, int lo, int hi) {
        for (int c0 = 0; c0 < E; c0 += kSoloThreads) {
            const int j = c0 + tid;
            int e = 0, base = 0, len = 0;
            uint64_t key = 0;
            if (j < E) {
                edge_of(in, r, j, e, base, len);
                key = solo_key(g, s, (int)e0 + e, r, rekey);
            }
            int total;
            const int st = solo_exclusive_sum(len, C.wave_tmp, &total);
            C.start[tid] = st;
            C.base[tid] = base;
            C.key[tid] = key;
            __syncthreads();
            scatter(total, lo, hi);
            __syncthreads();
        }
    };
    auto clear_tile = [&](int n) {
        for (int v = tid; v < n; v += kSoloThreads) best[v] = 0;
        __syncthreads();
    };

    if (one) {  // round 0's maximum: every edge at every pin
        clear_tile(nv);
        max_pass(list0, 0, ne, 0, nv);
    } else {
        __syncthreads();
    }
    int E = ne;
    unsigned long long K = (unsigned long long)(a.pin_base[inst + 1] - a.pin_base[inst]);
    unsigned long long tot_m = 0, tot_w = 0;  // the instance's matched edges and weight
    int r = 0;
    for (;;) {
        const int32_t *in = (r & 1) ? list1 : list0;
        nm = wm = pm = 0;
        if (one) {
            // ---- test: the first pin per lane (most edges fail there), the
            // remaining pins of the undecided edges spread over the workgroup
            for (int c0 = 0; c0 < E; c0 += kSoloThreads) {
                const int j = c0 + tid;
                int e = -1, base = 0, len = 0;
                uint64_t key = 0;
                bool ok = false;
                if (j < E) {
                    edge_of(in, r, j, e, base, len);
                    key = solo_key(g, s, (int)e0 + e, r, rekey);
                    ok = len == 0 || best[e_pins[base]] == key;
                }
                int total;
                const int st = solo_exclusive_sum(ok && len > 1 ? len - 1 : 0, C.wave_tmp, &total);
                if (total > 0) {
                    C.start[tid] = st;
                    C.base[tid] = base + 1;
                    C.key[tid] = key;
                    C.flag[tid] = 0;
                    __syncthreads();
                    for (int t0 = tid; t0 < total; t0 += kUnroll * kSoloThreads) {
                        int jj[kUnroll], pin[kUnroll];
                        solo_pins(C, e_pins, total, t0, jj, pin);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            if (jj[u] >= 0 && best[pin[u]] != C.key[jj[u]]) C.flag[jj[u]] = 1;
                    }
                    __syncthreads();
                    ok = ok && !C.flag[tid];
                    __syncthreads();
                }
                if (ok) record(e, base, len, key);
            }
        } else {
            // ---- maximum and test tile by tile
            for (int j = tid; j < E; j += kSoloThreads) fail[j] = 0;
            for (int t = 0; t < tiles; ++t) {
                const int lo = t * tile, hi = min(nv, lo + tile);
                clear_tile(hi - lo);
                max_pass(in, r, E, lo, hi);
                for (int c0 = 0; c0 < E; c0 += kSoloThreads) {
                    const int j = c0 + tid;
                    int e = 0, base = 0, len = 0;
                    uint64_t key = 0;
                    if (j < E) {
                        edge_of(in, r, j, e, base, len);
                        key = solo_key(g, s, (int)e0 + e, r, rekey);
                    }
                    int total;
                    const int st = solo_exclusive_sum(len, C.wave_tmp, &total);
                    C.start[tid] = st;
                    C.base[tid] = base;
                    C.key[tid] = key;
                    C.flag[tid] = 0;
                    __syncthreads();
                    for (int t0 = tid; t0 < total; t0 += kUnroll * kSoloThreads) {
                        int jj[kUnroll], pin[kUnroll];
                        solo_pins(C, e_pins, total, t0, jj, pin);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            if (jj[u] >= 0 && pin[u] >= lo && pin[u] < hi &&
                                best[pin[u] - lo] != C.key[jj[u]])
                                C.flag[jj[u]] = 1;
                    }
                    __syncthreads();
                    if (j < E && C.flag[tid]) fail[j] = 1;
                    __syncthreads();
                }
            }
            for (int j = tid; j < E; j += kSoloThreads) {
                if (fail[j]) continue;
                int e, base, len;
                edge_of(in, r, j, e, base, len);
                record(e, base, len, solo_key(g, s, (int)e0 + e, r, rekey));
            }
        }
        nm = solo_sum(nm, C.sum_tmp);
        wm = solo_sum(wm, C.sum_tmp);
        pm = solo_sum(pm, C.sum_tmp);
        tot_m += nm;
        tot_w += wm;
        if (tid == 0 && r < s.solo_rounds) {
            unsigned long long *row = s.solo + kSoloHeader + 5 * (int64_t)r;
            atomicAdd(&row[0], (unsigned long long)E);
            atomicAdd(&row[1], K);
            if (nm) {
                atomicAdd(&row[2], nm);
                atomicAdd(&row[3], wm);
                atomicAdd(&row[4], pm);
            }
        }
        // ---- clear the maximum for the next round (one tile; the test's
        // reads are done); the done marks are complete after the barrier
        if (one)
            clear_tile(nv);
        else
            __syncthreads();
        // ---- retire and compaction (with one tile also the next maximum)
        const int rn = r + 1;
        int32_t *out = (rn & 1) ? list1 : list0;
        int kept = 0;
        unsigned long long kn = 0;
        for (int c0 = 0; c0 < E; c0 += kSoloThreads) {
            const int j = c0 + tid;
            int e = -1, base = 0, len = 0;
            bool dead = true;
            if (j < E) {
                edge_of(in, r, j, e, base, len);
                dead = len == 0;  // an empty edge was matched by its test
                int p[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) p[u] = u < len ? e_pins[base + u] : -1;
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) dead = dead || (p[u] >= 0 && bit_is_set(done, p[u]));
            }
            int total;
            const int st = solo_exclusive_sum(!dead && len > kUnroll ? len - kUnroll : 0,
                                              C.wave_tmp, &total);
            if (total > 0) {
                C.start[tid] = st;
                C.base[tid] = base + kUnroll;
                C.flag[tid] = 0;
                __syncthreads();
                for (int t0 = tid; t0 < total; t0 += kUnroll * kSoloThreads) {
                    int jj[kUnroll], pin[kUnroll];
                    solo_pins(C, e_pins, total, t0, jj, pin);
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (jj[u] >= 0 && bit_is_set(done, pin[u])) C.flag[jj[u]] = 1;
                }
                __syncthreads();
                dead = dead || C.flag[tid];
                __syncthreads();
            }
            const bool alive = !dead;
            int n_alive;
            const int pos = solo_exclusive_sum(alive ? 1 : 0, C.wave_tmp, &n_alive);
            int total2;
            const int st2 = solo_exclusive_sum(alive ? len : 0, C.wave_tmp, &total2);
            if (alive) out[kept + pos] = e;
            if (one) {
                C.start[tid] = st2;
                C.base[tid] = base;
                C.key[tid] = alive ? solo_key(g, s, (int)e0 + e, rn, rekey) : 0;
                __syncthreads();
                scatter(total2, 0, nv);
                __syncthreads();
            }
            kept += n_alive;
            kn += (unsigned long long)total2;
        }
        K = kn;
        E = kept;
        r = rn;
        if (E == 0) break;
        if (a.max_rounds > 0 && r >= a.max_rounds) {
            if (tid == 0) atomicOr(&s.solo[1], 1ull);
            break;
        }
    }
    if (tid == 0) {
        atomicMax(&s.solo[0], (unsigned long long)r);
        if (tot_m) {
            atomicAdd(&s.solo[3], tot_m);
            atomicAdd(&s.solo[4], tot_w);
        }
    }
    // The instance is finished for the round kernels: every vertex done, so
    // the vertex-centric passes of the batch skip it.
    for (int v = tid; v < nv; v += kSoloThreads) s.done[v0 + v] = 1;
    __syncthreads();
}

// Instances are taken largest-first in two sweeps of one counter: sweep 0
// takes the instances that need several LDS tiles, sweep 1 the others, so
// the longest ones do not start last.
__global__ void __launch_bounds__(kSoloThreads) k_solo(Graph g, State s, SoloArgs a,
                                                       uint32_t *bits, int rekey) {
    extern __shared__ unsigned char solo_lds[];
    __shared__ SoloChunk C;
    for (;;) {
        if (threadIdx.x == 0) C.inst = (int)atomicAdd(&s.solo[2], 1ull);
        __syncthreads();
        const int q = C.inst;
        __syncthreads();  // every thread has read the index before it is overwritten
        if (q >= 2 * a.count) break;
        const int i = q < a.count ? q : q - a.count;
        if (!solo_instance(a.v_base[i + 1] - a.v_base[i], a.pin_base[i + 1] - a.pin_base[i], a))
            continue;
        if (a.e_base[i + 1] == a.e_base[i]) continue;  // no edges: nothing to match
        const bool big = a.v_base[i + 1] - a.v_base[i] > a.one_tile;
        if (big != (q < a.count)) continue;
        solo_run(g, s, a, bits, rekey != 0, i, solo_lds, C);
    }
}

// Round 0's explicit live list for the round kernels: the edges of the
// instances outside the solo part, with their records (pin offset, count,
// first pin, vertex base, key), spread evenly over the workgroups' regions
// in edge order (the rounds' cost follows the fullest region, and the solo
// part leaves the remaining edges unevenly spread over the id range).  Two
// passes: each workgroup counts the kept edges of its own id range into
// cnt[1] (free until round 1's retire), then places them by global rank.
__device__ __forceinline__ bool live0_keep(const SoloArgs &a, int &i, int64_t e) {
    while (i + 1 < a.count && a.e_base[i + 1] <= e) ++i;
    return !solo_instance(a.v_base[i + 1] - a.v_base[i], a.pin_base[i + 1] - a.pin_base[i], a);
}

__global__ void __launch_bounds__(kBlock) k_live0_count(Graph g, State s, SoloArgs a) {
    __shared__ int first;
    __shared__ unsigned long long sum_tmp[kWaves];
    const int b = xcd_item(blockIdx.x, gridDim.x);
    const int64_t lo = (int64_t)b * s.region;
    const int64_t hi = lo + s.region < (int64_t)g.m ? lo + s.region : (int64_t)g.m;
    unsigned long long kept = 0;
    if (lo < hi) {
        if (threadIdx.x == 0) first = instance_of(a.e_base, a.count, lo);
        __syncthreads();
        int i = first;
        for (int64_t e = lo + threadIdx.x; e < hi; e += kBlock) kept += live0_keep(a, i, e) ? 1 : 0;
    }
    kept = block_sum_u64(kept, sum_tmp);
    if (threadIdx.x == 0) s.cnt[1][b] = (int)kept;
}

__global__ void __launch_bounds__(kBlock) k_live0_place(Graph g, State s, SoloArgs a) {
    __shared__ int first;
    __shared__ int wave_tmp[kWaves];
    __shared__ unsigned long long sum_tmp[kWaves];
    const int b = xcd_item(blockIdx.x, gridDim.x);
    // Kept edges before this workgroup's range, and in all.
    unsigned long long before = 0, all = 0;
    for (int q = threadIdx.x; q < s.grid; q += kBlock) {
        const unsigned long long c = (unsigned long long)s.cnt[1][q];
        all += c;
        before += q < b ? c : 0;
    }
    before = block_sum_u64(before, sum_tmp);
    all = block_sum_u64(all, sum_tmp);
    const int64_t per = ((int64_t)all + s.grid - 1) / s.grid;  // <= region (all <= m)
    const int64_t lo = (int64_t)b * s.region;
    const int64_t hi = lo + s.region < (int64_t)g.m ? lo + s.region : (int64_t)g.m;
    unsigned long long kap = 0;
    int64_t rank = (int64_t)before;
    if (lo < hi) {
        if (threadIdx.x == 0) first = instance_of(a.e_base, a.count, lo);
        __syncthreads();
        int i = first;
        for (int64_t c0 = lo; c0 < hi; c0 += kBlock) {
            const int64_t e = c0 + threadIdx.x;
            const bool keep = e < hi && live0_keep(a, i, e);
            int total;
            const int pos = block_exclusive_sum(keep ? 1 : 0, wave_tmp, &total);
            if (keep) {
                const int64_t q = rank + pos;
                const int64_t at = (q / per) * s.region + q % per;
                const int base = g.e_off[e], len = g.e_off[e + 1] - base;
                const int vb = g.vbase[e];
                s.list[0][at] = (int)e;
                s.rec_a[0][at] = base;
                s.rec_b[0][at] = len;
                s.rec_c[0][at] = len > 0 ? g.e_pins[base] + vb : -1;
                s.rec_vb[0][at] = vb;
                s.rec_key[0][at] = s.key[e];
                kap += (unsigned long long)len;
            }
            rank += total;
        }
    }
    kap = block_sum_u64(kap, sum_tmp);
    if (threadIdx.x == 0) {
        const int64_t mine = (int64_t)all - (int64_t)b * per;
        s.cnt[0][b] = (int)(mine <= 0 ? 0 : mine < per ? mine : per);
        if (kap > 0) atomicAdd(&s.stats[0].kappa[b % kSub], kap);
        if (b == 0 && all > 0) atomicAdd(&s.stats[0].live[0], all);
    }
}

// ---------------------------------------------------------------------------
// Tail of one instance.  Late rounds have few live edges, and three
// grid-wide launches per round then cost far more than their work.  After
// the retire pass of round R, one workgroup reads R's live counts; when
// they are within the tail's bounds it gathers every workgroup's live list
// (with its records) into one compact list, empties the lists so that the
// rounds still enqueued after it find nothing to do, and runs rounds R,
// R + 1, ... itself until no live edge remains (or max_rounds is reached):
//   test    a live edge whose key equals best at every pin is matched; its
//           bit is set and its pins marked done
//   retire  every other live edge with a done pin leaves; the survivors
//           are compacted into the other list with their next-round key
//   max     best of the next round: zero at the survivors' pins, then each
//           survivor raises it at its pins
// best[R & 1] already holds round R's maximum (the retire pass of R built
// it).  Counters of each round go to the tail record.  Each lane handles
// kTailU list slots per step, their loads issued together.
constexpr int kTailWaves = kTailThreads / kWave;
constexpr int kTailU = 8;

__device__ __forceinline__ int tail_exclusive_sum(int v, int *wave_tmp, int *total) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) wave_tmp[wid] = incl;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kTailWaves; ++i) {
        const int x = wave_tmp[i];
        off += (i < wid) ? x : 0;
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return off + incl - v;
}

__device__ __forceinline__ unsigned long long tail_sum(unsigned long long v,
                                                       unsigned long long *tmp) {
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) tmp[wid] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int i = 0; i < kTailWaves; ++i) t += tmp[i];
    __syncthreads();
    return t;
}

// Pin k of a tail slot: pair layout (a, b) are the two pins; offset layout
// a = pin offset, b = count.
__device__ __forceinline__ int tail_pin(const Graph &g, int a, int b, int k) {
    return g.pairs ? (k == 0 ? a : b) : g.e_pins[a + k];
}

__device__ __forceinline__ int tail_len(const Graph &g, int b) { return g.pairs ? 2 : b; }

__global__ void __launch_bounds__(kTailThreads) k_tail(Graph g, State s, int round,
                                                       uint32_t *bits, uint32_t seed,
                                                       int reseed, int max_rounds) {
    __shared__ int wave_tmp[kTailWaves];
    __shared__ unsigned long long sum_tmp[kTailWaves];
    __shared__ int take;
    const int tid = threadIdx.x;
    if (s.tail[0] != 0) return;  // an earlier launch took over (uniform read)
    if (tid < kWave) {
        const RoundStats &st = s.stats[round % s.ring];
        unsigned long long live = st.live[tid], kap = st.kappa[tid];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            live += __shfl_xor(live, o, kWave);
            kap += __shfl_xor(kap, o, kWave);
        }
        if (tid == 0)
            take = live > 0 && live <= (unsigned long long)s.tail_cap &&
                   kap <= (unsigned long long)s.tail_pins;
    }
    __syncthreads();
    if (!take || (max_rounds > 0 && round >= max_rounds)) return;
    // Gather the workgroups' live lists of `round` into tail list 0.
    const int k = round & 1;
    int E = 0;
    unsigned long long K = 0;
    for (int c0 = 0; c0 < s.grid; c0 += kTailThreads) {
        const int b = c0 + tid;
        const int n = b < s.grid ? s.cnt[k][b] : 0;
        int total;
        const int at = E + tail_exclusive_sum(n, wave_tmp, &total);
        for (int i = 0; i < n; ++i) {
            const int64_t src = (int64_t)b * s.region + i;
            s.tail_e[0][at + i] = s.list[k][src];
            s.tail_a[0][at + i] = s.rec_a[k][src];
            s.tail_b[0][at + i] = s.rec_b[k][src];
            s.tail_key[0][at + i] = s.rec_key[k][src];
            K += (unsigned long long)tail_len(g, s.rec_b[k][src]);
        }
        if (b < s.grid) {
            s.cnt[k][b] = 0;
            s.cnt[k ^ 1][b] = 0;
        }
        E += total;
    }
    K = tail_sum(K, sum_tmp);
    __syncthreads();  // the gathered list is complete
    const int e0 = E;  // every round matches at least its largest live edge
    int r = round, p = 0;
    unsigned long long *rows = s.tail + kTailHeader;
    for (;;) {
        const uint64_t *best = s.best[r & 1];
        // ---- test
        unsigned long long nm = 0, wm = 0, pm = 0;
        for (int j0 = tid; j0 < E; j0 += kTailU * kTailThreads) {
            int a[kTailU], bb[kTailU], e[kTailU], pin0[kTailU];
            uint64_t key[kTailU], bv[kTailU];
#pragma unroll
            for (int u = 0; u < kTailU; ++u) {
                const int j = j0 + u * kTailThreads;
                const bool v = j < E;
                e[u] = v ? s.tail_e[p][j] : -1;
                a[u] = v ? s.tail_a[p][j] : 0;
                bb[u] = v ? s.tail_b[p][j] : 0;
                key[u] = v ? s.tail_key[p][j] : 0;
            }
#pragma unroll
            for (int u = 0; u < kTailU; ++u)
                pin0[u] = (e[u] >= 0 && tail_len(g, bb[u]) > 0) ? tail_pin(g, a[u], bb[u], 0) : -1;
#pragma unroll
            for (int u = 0; u < kTailU; ++u)
                bv[u] = pin0[u] >= 0 ? __hip_atomic_load(&best[pin0[u]], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP)
                                     : key[u];
#pragma unroll
            for (int u = 0; u < kTailU; ++u) {
                if (e[u] < 0) continue;
                const int len = tail_len(g, bb[u]);
                bool ok = bv[u] == key[u];
                for (int q = 1; q < len && ok; ++q)
                    ok = __hip_atomic_load(&best[tail_pin(g, a[u], bb[u], q)], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP) == key[u];
                if (!ok) continue;
                atomicOr(&bits[e[u] >> 5], 1u << (e[u] & 31));
                nm += 1;
                wm += key[u] >> 32;
                pm += (unsigned long long)len;
                for (int q = 0; q < len; ++q) s.done[tail_pin(g, a[u], bb[u], q)] = 1;
            }
        }
        nm = tail_sum(nm, sum_tmp);
        wm = tail_sum(wm, sum_tmp);
        pm = tail_sum(pm, sum_tmp);
        if (tid == 0) {
            unsigned long long *row = rows + 5 * (int64_t)(r - round);
            row[0] = (unsigned long long)E;
            row[1] = K;
            row[2] = nm;
            row[3] = wm;
            row[4] = pm;
        }
        // ---- retire and compaction (the done marks are complete: the sums
        // above end with a barrier)
        const int rn = r + 1;
        const uint32_t kseed_next = reseed ? round_seed(seed, rn) : seed;
        int kept = 0;
        unsigned long long kn = 0;
        for (int c0 = 0; c0 < E; c0 += kTailU * kTailThreads) {
            int a[kTailU], bb[kTailU], e[kTailU];
            uint64_t key[kTailU];
            bool alive[kTailU];
            int mine = 0;
#pragma unroll
            for (int u = 0; u < kTailU; ++u) {
                const int j = c0 + tid * kTailU + u;  // lane-contiguous slots: kept in order
                const bool v = j < E;
                e[u] = v ? s.tail_e[p][j] : -1;
                a[u] = v ? s.tail_a[p][j] : 0;
                bb[u] = v ? s.tail_b[p][j] : 0;
                key[u] = v ? s.tail_key[p][j] : 0;
            }
#pragma unroll
            for (int u = 0; u < kTailU; ++u) {
                const int len = e[u] >= 0 ? tail_len(g, bb[u]) : 0;
                bool dead = e[u] < 0 || len == 0;  // an empty edge was matched by its test
                for (int q = 0; q < len && !dead; ++q) dead = s.done[tail_pin(g, a[u], bb[u], q)] != 0;
                alive[u] = !dead;
                mine += alive[u] ? 1 : 0;
            }
            int total;
            int at = kept + tail_exclusive_sum(mine, wave_tmp, &total);
#pragma unroll
            for (int u = 0; u < kTailU; ++u) {
                if (!alive[u]) continue;
                s.tail_e[p ^ 1][at] = e[u];
                s.tail_a[p ^ 1][at] = a[u];
                s.tail_b[p ^ 1][at] = bb[u];
                s.tail_key[p ^ 1][at] =
                    reseed ? edge_key<false>(g, s, kseed_next, e[u]) : key[u];
                kn += (unsigned long long)tail_len(g, bb[u]);
                ++at;
            }
            kept += total;
        }
        K = tail_sum(kn, sum_tmp);  // ends with a barrier: the new list is complete
        E = kept;
        r = rn;
        p ^= 1;
        if (E == 0) break;
        if (max_rounds > 0 && r >= max_rounds) {
            if (tid == 0) s.tail[2] = 1;
            break;
        }
        if (r - round >= e0) {  // cannot happen with a correct maximum: stop, reported
            if (tid == 0) s.tail[2] = 2;
            break;
        }
        // ---- the next round's maximum: zero at the survivors' pins, then raise
        uint64_t *nb = s.best[r & 1];
        for (int j = tid; j < E; j += kTailThreads) {
            const int a = s.tail_a[p][j], bb = s.tail_b[p][j], len = tail_len(g, bb);
            for (int q = 0; q < len; ++q) nb[tail_pin(g, a, bb, q)] = 0;
        }
        __syncthreads();
        for (int j = tid; j < E; j += kTailThreads) {
            const int a = s.tail_a[p][j], bb = s.tail_b[p][j], len = tail_len(g, bb);
            const uint64_t key = s.tail_key[p][j];
            for (int q = 0; q < len; ++q)
                __hip_atomic_fetch_max(&nb[tail_pin(g, a, bb, q)], key, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
    }
    if (tid == 0) {
        s.tail[1] = (unsigned long long)r;
        s.tail[0] = (unsigned long long)round + 1;
    }
}

__global__ void __launch_bounds__(kBlock) k_zero_words(uint32_t *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

}  // namespace

hipError_t launch_init(const Launch &L, const Graph &g, uint32_t seed, const State &s,
                       uint32_t *bits, int init_flags) {
    hipLaunchKernelGGL(k_prologue, dim3(1), dim3(kBlock), 0, L.stream, g, s);
    hipLaunchKernelGGL(k_init, dim3(L.grid), dim3(kBlock), 0, L.stream, g, seed, s, bits,
                       init_flags);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const Launch &L, const Graph &g, const BatchIn &b, const State &s) {
    if (b.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_setup, dim3(L.grid), dim3(kBlock), 0, L.stream, g, b, s);
    return hipGetLastError();
}

hipError_t launch_solo(const Launch &L, const Graph &g, const State &s, const SoloArgs &a,
                       uint32_t *bits, int rekey, int workgroups) {
    const size_t lds = (size_t)a.lds_bytes;
    static std::atomic<size_t> granted{0};
    if (granted.load(std::memory_order_relaxed) < lds) {
        hipError_t rc = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_solo),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (rc != hipSuccess) return rc;
        granted.store(lds, std::memory_order_relaxed);
    }
    hipLaunchKernelGGL(k_solo, dim3(workgroups), dim3(kSoloThreads), lds, L.stream, g, s, a, bits,
                       rekey);
    return hipGetLastError();
}

hipError_t launch_live0(const Launch &L, const Graph &g, const State &s, const SoloArgs &a) {
    hipLaunchKernelGGL(k_live0_count, dim3(s.grid), dim3(kBlock), 0, L.stream, g, s, a);
    hipLaunchKernelGGL(k_live0_place, dim3(s.grid), dim3(kBlock), 0, L.stream, g, s, a);
    return hipGetLastError();
}

hipError_t launch_tail(const Launch &L, const Graph &g, const State &s, int round,
                       uint32_t *bits, uint32_t seed, int reseed, int max_rounds) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), 0, L.stream, g, s, round, bits, seed,
                       reseed, max_rounds);
    return hipGetLastError();
}

hipError_t launch_validate(const Launch &L, const Graph &g, const State &s, int check_dual) {
    if (check_dual)
        hipLaunchKernelGGL(k_zero_words, dim3(L.grid), dim3(kBlock), 0, L.stream, s.vbits,
                           (g.kappa + 31) / 32);
    hipLaunchKernelGGL(k_validate, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s, check_dual);
    return hipGetLastError();
}

// Launch helpers: the instantiation follows the layout (graph pairs or
// offsets) and whether the graph is a batch (g.vbase set); batches of graphs
// in the pair layout are rejected by the interface.
hipError_t launch_scatter(const Launch &L, const Graph &g, const State &s, uint32_t kseed) {
    const dim3 grid(s.grid), block(kBlock);
    if (g.pairs)
        hipLaunchKernelGGL((k_scatter0<true, false>), grid, block, 0, L.stream, g, s, kseed);
    else if (g.vbase)
        hipLaunchKernelGGL((k_scatter0<false, true>), grid, block, 0, L.stream, g, s, kseed);
    else
        hipLaunchKernelGGL((k_scatter0<false, false>), grid, block, 0, L.stream, g, s, kseed);
    return hipGetLastError();
}

hipError_t launch_retire(const Launch &L, const Graph &g, const State &s, int round, int scatter,
                         uint32_t kseed, int rekey, int binned) {
    const dim3 grid(s.grid), block(kBlock);
    if (binned) {
        if (!scatter || g.pairs || g.vbase || s.bin_nb <= 0 || s.bin_nb > kBinMaxBins ||
            s.bin_rb < kBinMinShift || s.bin_rb > kBinMaxShift || !g.v_off)
            return hipErrorInvalidValue;
        const size_t tile = (size_t)8 << s.bin_rb;
        static std::atomic<size_t> granted{0};
        if (granted.load(std::memory_order_relaxed) < tile) {
            hipError_t rc = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bin_max),
                                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)tile);
            if (rc != hipSuccess) return rc;
            granted.store(tile, std::memory_order_relaxed);
        }
        hipLaunchKernelGGL(k_retire_bin, grid, block, 8 * (size_t)s.bin_nb, L.stream, g, s, round,
                           kseed, rekey);
        hipLaunchKernelGGL(k_bin_max, dim3(s.bin_nb), dim3(kBinThreads), tile, L.stream, g, s,
                           round);
        return hipGetLastError();
    }
#define HGM_RETIRE(P, S, B) \
    hipLaunchKernelGGL((k_retire<P, S, B>), grid, block, 0, L.stream, g, s, round, kseed, rekey)
    if (g.pairs) {
        if (scatter) HGM_RETIRE(true, true, false);
        else HGM_RETIRE(true, false, false);
    } else if (g.vbase) {
        if (scatter) HGM_RETIRE(false, true, true);
        else HGM_RETIRE(false, false, true);
    } else {
        if (scatter) HGM_RETIRE(false, true, false);
        else HGM_RETIRE(false, false, false);
    }
#undef HGM_RETIRE
    return hipGetLastError();
}

hipError_t launch_max0(const Launch &L, const Graph &g, const State &s, uint32_t seed) {
    const dim3 eg(s.grid), vg(L.grid), block(kBlock);
    if (g.pairs)
        hipLaunchKernelGGL((k_max0_edge<true, false>), eg, block, 0, L.stream, g, s, seed);
    else if (g.vbase)
        hipLaunchKernelGGL((k_max0_edge<false, true>), eg, block, 0, L.stream, g, s, seed);
    else
        hipLaunchKernelGGL((k_max0_edge<false, false>), eg, block, 0, L.stream, g, s, seed);
    if (g.vbase)
        hipLaunchKernelGGL(k_max0_vertex<true>, vg, block, 0, L.stream, g, s, seed);
    else
        hipLaunchKernelGGL(k_max0_vertex<false>, vg, block, 0, L.stream, g, s, seed);
    return hipGetLastError();
}

hipError_t launch_vertex_max(const Launch &L, const Graph &g, const State &s, int round,
                             uint32_t kseed, int rekey) {
    const dim3 grid(L.grid), block(kBlock);
    if (g.vbase)
        hipLaunchKernelGGL(k_vertex_max<true>, grid, block, 0, L.stream, g, s, round, kseed, rekey);
    else
        hipLaunchKernelGGL(k_vertex_max<false>, grid, block, 0, L.stream, g, s, round, kseed,
                           rekey);
    return hipGetLastError();
}

hipError_t launch_test(const Launch &L, const Graph &g, const State &s, int round, int clear,
                       uint32_t *bits, uint32_t kseed) {
    const dim3 grid(s.grid), block(kBlock);
#define HGM_TEST(P, C, B) \
    hipLaunchKernelGGL((k_test<P, C, B>), grid, block, 0, L.stream, g, s, round, bits, kseed)
#define HGM_TEST_CLEAR(P, B)                                        \
    do {                                                            \
        if (clear == kClearAll) HGM_TEST(P, kClearAll, B);          \
        else if (clear == kClearPins) HGM_TEST(P, kClearPins, B);   \
        else HGM_TEST(P, kClearNone, B);                            \
    } while (0)
    if (g.pairs) HGM_TEST_CLEAR(true, false);
    else if (g.vbase) HGM_TEST_CLEAR(false, true);
    else HGM_TEST_CLEAR(false, false);
#undef HGM_TEST_CLEAR
#undef HGM_TEST
    return hipGetLastError();
}

}  // namespace hgm
