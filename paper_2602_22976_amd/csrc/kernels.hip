// Round kernels of iterated local-max hypergraph matching for gfx950.
//
// One round of the method (paper, Section 4.1 and Algorithms 1/2):
//   max    every vertex v takes best[v] = max key over its live incident edges
//   test   a live edge e whose key equals best[v] at every pin v is matched;
//          its pins are marked done
//   retire every live edge with a done pin leaves the live set (soft delete)
// Keys are fixed: key(e) = w(e) << 32 | H(seed, e), with H = MurmurHash3_x86_32
// of e's little-endian bytes; H is a bijection, so keys are distinct.
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
// Round r uses list[r & 1] (round 0 uses the identity list 0..m-1) and the
// counters slots[r % ring].  best[] is double-buffered by round parity so that
// the test of round r can clear the buffer round r+1 will fill.
#include "internal.h"

namespace hgm {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) {
    return (x << r) | (x >> (32 - r));
}

// MurmurHash3_x86_32 (Appleby) of the four little-endian bytes of `id`:
// one body block, no tail, length 4, then the fmix32 finaliser.
__device__ __forceinline__ uint32_t priority_hash(uint32_t seed, uint32_t id) {
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

__device__ __forceinline__ int wave_inclusive_sum(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
    }
    return v;
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

// Largest j in [0, kBlock) with start[j] <= t (start non-decreasing, start[0] = 0).
__device__ __forceinline__ int find_item(const int *start, int t) {
    int j = 0;
#pragma unroll
    for (int step = kBlock / 2; step > 0; step >>= 1)
        if (start[j + step] <= t) j += step;
    return j;
}

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    int wave_tmp[kWaves];
    unsigned long long sum_tmp[kWaves];
    int out_base;
};

// ---------------------------------------------------------------------------
// Setup: keys, cleared per-vertex state, cleared bitmap, round-0 counters.
__global__ void __launch_bounds__(kBlock) k_init(Graph g, uint32_t seed, State s, uint32_t *bits,
                                                 int crew) {
    const int64_t words = ((int64_t)g.m + 31) / 32;
    const int64_t span = g.m > g.n ? g.m : g.n;
    const int64_t top = span > words ? span : words;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < top; i += stride) {
        if (i < g.m) {
            uint64_t k = ((uint64_t)g.w[i] << 32) | priority_hash(seed, (uint32_t)i);
            s.key[i] = k;
            if (crew) s.live_key[i] = k;
        }
        if (i < g.n) {
            s.best[0][i] = 0;
            s.done[i] = 0;
        }
        if (i < words) bits[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < s.ring) {
        RoundSlot z = {0, 0, 0, 0, 0};
        if (threadIdx.x == 0) {
            z.live = g.m;
            z.kappa = g.m > 0 ? g.e_off[g.m] : 0;
        }
        s.slots[threadIdx.x] = z;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *s.err = 0;
        if (crew) *s.hub_count = 0;
    }
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
    if (tid0 == 0) {
        if (g.m > 0 && (g.e_off[0] != 0 || g.e_off[g.m] != kap)) atomicOr(s.err, 1);
        if (check_dual && (g.v_off[0] != 0 || g.v_off[g.n] != kap)) atomicOr(s.err, 2);
    }
    for (int64_t e = tid0; e < g.m; e += stride) {
        int32_t a = g.e_off[e], b = g.e_off[e + 1];
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
            int32_t ea = g.e_off[e], eb = g.e_off[e + 1];
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
// Edge-centric scatter of round 0 (Algorithm 1, per-vertex maximum by
// concurrent writes): every edge raises best[pin] to its key at each pin.
// The plain read first skips the atomic when the slot already holds a larger
// key; best only grows during the pass, so a stale read is merely cautious.
__global__ void __launch_bounds__(kBlock) k_scatter0(Graph g, State s) {
    __shared__ ChunkLds L;
    uint64_t *best = s.best[0];
    const int m = g.m;
    for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < m; c0 += (int64_t)gridDim.x * kBlock) {
        const int i = (int)c0 + threadIdx.x;
        int len = 0, base = 0;
        uint64_t key = 0;
        if (i < m) {
            base = g.e_off[i];
            len = g.e_off[i + 1] - base;
            key = s.key[i];
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        __syncthreads();
        for (int t = threadIdx.x; t < total; t += kBlock) {
            int j = find_item(L.start, t);
            int pin = g.e_pins[L.base[j] + (t - L.start[j])];
            uint64_t k = L.key[j];
            if (load_relaxed(&best[pin]) < k) atomic_max_u64(&best[pin], k);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Retire + compact (+ scatter) for round r >= 1.  Input: the live list of
// round r-1 (identity for r-1 = 0) and its count.  An edge of that list
// survives iff it is non-empty and none of its pins is done; this removes the
// edges matched in round r-1 (all their pins are done) and every edge that
// touches them (Algorithm 2's OR-reduction over the pins of each edge).
// Survivors are appended to list[r & 1] (one atomic per chunk) and counted
// into slots[r].  Then, depending on the variant:
//   scatter = 1 (CRCW): each survivor raises best[r & 1][pin] at its pins.
//   scatter = 0 (CREW): non-survivors get live_key = 0, and the split hub
//                       vertices' best[r & 1] is cleared for the vertex pass.
__global__ void __launch_bounds__(kBlock) k_retire(Graph g, State s, int round, int scatter) {
    __shared__ ChunkLds L;
    const RoundSlot *in_slot = &s.slots[(round - 1) % s.ring];
    RoundSlot *out_slot = &s.slots[round % s.ring];
    const int32_t *in_list = (round - 1 == 0) ? nullptr : s.list[(round - 1) & 1];
    int32_t *out_list = s.list[round & 1];
    uint64_t *best = s.best[round & 1];
    const int cnt = in_slot->live;

    if (!scatter && blockIdx.x == 0) {
        const int h = *s.hub_count;
        for (int i = threadIdx.x; i < h; i += kBlock) best[s.hubs[i]] = 0;
    }
    for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < cnt; c0 += (int64_t)gridDim.x * kBlock) {
        const int i = (int)c0 + threadIdx.x;
        int e = -1, len = 0, base = 0;
        uint64_t key = 0;
        if (i < cnt) {
            e = in_list ? in_list[i] : i;
            base = g.e_off[e];
            len = g.e_off[e + 1] - base;
            key = s.key[e];
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        L.flag[threadIdx.x] = 0;
        __syncthreads();
        for (int t = threadIdx.x; t < total; t += kBlock) {
            int j = find_item(L.start, t);
            int pin = g.e_pins[L.base[j] + (t - L.start[j])];
            if (s.done[pin]) L.flag[j] = 1;
        }
        __syncthreads();
        const int alive = (e >= 0 && len > 0 && !L.flag[threadIdx.x]) ? 1 : 0;
        if (!scatter && e >= 0 && !alive) s.live_key[e] = 0;
        int n_alive;
        int pos = block_exclusive_sum(alive, L.wave_tmp, &n_alive);
        unsigned long long kap = block_sum_u64(alive ? (unsigned long long)len : 0ull, L.sum_tmp);
        if (threadIdx.x == 0 && n_alive > 0) {
            L.out_base = atomicAdd(&out_slot->live, n_alive);
            atomicAdd((unsigned long long *)&out_slot->kappa, kap);
        }
        __syncthreads();
        if (alive) out_list[L.out_base + pos] = e;
        if (scatter) {
            int total2;
            int st2 = block_exclusive_sum(alive ? len : 0, L.wave_tmp, &total2);
            L.start[threadIdx.x] = st2;
            __syncthreads();
            for (int t = threadIdx.x; t < total2; t += kBlock) {
                int j = find_item(L.start, t);
                int pin = g.e_pins[L.base[j] + (t - L.start[j])];
                uint64_t k = L.key[j];
                if (load_relaxed(&best[pin]) < k) atomic_max_u64(&best[pin], k);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Vertex-centric maximum of round r (Algorithm 2, segmented MAX over each
// vertex's incidence list).  Chunks of kBlock consecutive vertices: done
// vertices and split hubs contribute no incidences; the chunk's incidences
// are flattened over the lanes, each wave reduces runs of equal vertex with a
// segmented max-scan in registers, and one LDS atomic per run and wave
// combines the runs.  Hubs (degree > hub_threshold) are cut into pieces of
// kHubPiece incidences, each reduced by one workgroup and combined with one
// global atomic max (their best was cleared by the retire pass).
constexpr int kHubPiece = 8192;

__global__ void __launch_bounds__(kBlock) k_vertex_max(Graph g, State s, int round, int hub_threshold) {
    __shared__ ChunkLds L;
    uint64_t *best = s.best[round & 1];
    const int lane = threadIdx.x & (kWave - 1);

    // Hub pieces first.  Piece q belongs to the hub h with
    // hub_piece_off[h] <= q < hub_piece_off[h+1] and covers kHubPiece
    // incidences of its list; pieces are spread over all workgroups.
    const int nh = *s.hub_count;
    const int n_pieces = nh > 0 ? s.hub_piece_off[nh] : 0;
    for (int q = blockIdx.x; q < n_pieces; q += gridDim.x) {
        int lo = 0, hi = nh - 1;  // last h with hub_piece_off[h] <= q
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s.hub_piece_off[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int v = s.hubs[lo];
        if (s.done[v]) continue;
        const int p0 = g.v_off[v] + (q - s.hub_piece_off[lo]) * kHubPiece;
        const int p1 = min(g.v_off[v + 1], p0 + kHubPiece);
        uint64_t mx = 0;
        for (int i = p0 + threadIdx.x; i < p1; i += kBlock) {
            uint64_t k = s.live_key[g.v_edges[i]];
            mx = k > mx ? k : mx;
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            uint64_t y = __shfl_xor(mx, o, kWave);
            mx = y > mx ? y : mx;
        }
        if (lane == 0 && mx) atomic_max_u64(&best[v], mx);
    }

    for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < g.n; c0 += (int64_t)gridDim.x * kBlock) {
        const int v = (int)c0 + threadIdx.x;
        int len = 0, base = 0;
        bool own = false;
        if (v < g.n && !s.done[v]) {
            base = g.v_off[v];
            len = g.v_off[v + 1] - base;
            own = len <= hub_threshold;
            if (!own) len = 0;
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = 0;
        __syncthreads();
        for (int t0 = 0; t0 < total; t0 += kBlock) {
            const int t = t0 + threadIdx.x;
            int j = -1;
            uint64_t k = 0;
            if (t < total) {
                j = find_item(L.start, t);
                k = s.live_key[g.v_edges[L.base[j] + (t - L.start[j])]];
            }
            // segmented inclusive max-scan over the wave, segments = equal j
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                uint64_t y = __shfl_up(k, o, kWave);
                int yj = __shfl_up(j, o, kWave);
                if (lane >= o && yj == j && y > k) k = y;
            }
            int nj = __shfl_down(j, 1, kWave);
            bool last = (lane == kWave - 1) || (nj != j);
            if (j >= 0 && last && k) atomicMax((unsigned long long *)&L.key[j], (unsigned long long)k);
        }
        __syncthreads();
        if (own) best[v] = L.key[threadIdx.x];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Local-max test of round r (Algorithm 1 third phase; Algorithm 2 P_e = |e|):
// a live edge is matched iff best[v] == key(e) at every pin v.  Matched edges
// set their bitmap bit and mark their pins done (exclusive: a vertex has one
// maximum edge).  With clear_next the pass also zeroes best[(r+1) & 1] at
// every pin it reads; the next round's survivors are a subset of this
// round's live edges, so the next scatter starts from zero at all its pins.
// The first thread also clears the counters of round r+1.
__global__ void __launch_bounds__(kBlock) k_test(Graph g, State s, int round, int clear_next,
                                                 uint32_t *bits) {
    __shared__ ChunkLds L;
    RoundSlot *slot = &s.slots[round % s.ring];
    const int32_t *list = round == 0 ? nullptr : s.list[round & 1];
    const uint64_t *best = s.best[round & 1];
    uint64_t *next = s.best[(round + 1) & 1];
    const int cnt = slot->live;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        RoundSlot z = {0, 0, 0, 0, 0};
        s.slots[(round + 1) % s.ring] = z;
    }
    for (int64_t c0 = (int64_t)blockIdx.x * kBlock; c0 < cnt; c0 += (int64_t)gridDim.x * kBlock) {
        const int i = (int)c0 + threadIdx.x;
        int e = -1, len = 0, base = 0;
        uint64_t key = 0;
        if (i < cnt) {
            e = list ? list[i] : i;
            base = g.e_off[e];
            len = g.e_off[e + 1] - base;
            key = s.key[e];
        }
        int total;
        int st = block_exclusive_sum(len, L.wave_tmp, &total);
        L.start[threadIdx.x] = st;
        L.base[threadIdx.x] = base;
        L.key[threadIdx.x] = key;
        L.flag[threadIdx.x] = 0;
        __syncthreads();
        for (int t = threadIdx.x; t < total; t += kBlock) {
            int j = find_item(L.start, t);
            int pin = g.e_pins[L.base[j] + (t - L.start[j])];
            if (best[pin] != L.key[j]) L.flag[j] = 1;
            if (clear_next) next[pin] = 0;
        }
        __syncthreads();
        const int matched = (e >= 0 && !L.flag[threadIdx.x]) ? 1 : 0;
        if (matched) atomicOr(&bits[e >> 5], 1u << (e & 31));
        unsigned long long nm = block_sum_u64(matched, L.sum_tmp);
        unsigned long long wm = block_sum_u64(matched ? (unsigned long long)(key >> 32) : 0ull,
                                              L.sum_tmp);
        if (threadIdx.x == 0 && nm) {
            atomicAdd((unsigned long long *)&slot->matched, nm);
            atomicAdd((unsigned long long *)&slot->weight, wm);
        }
        int total2;
        int st2 = block_exclusive_sum(matched ? len : 0, L.wave_tmp, &total2);
        L.start[threadIdx.x] = st2;
        __syncthreads();
        for (int t = threadIdx.x; t < total2; t += kBlock) {
            int j = find_item(L.start, t);
            s.done[g.e_pins[L.base[j] + (t - L.start[j])]] = 1;
        }
        __syncthreads();
    }
}

// Builds the list of split (hub) vertices for the vertex-centric pass.
__global__ void __launch_bounds__(kBlock) k_find_hubs(Graph g, State s, int hub_threshold) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        if (g.v_off[v + 1] - g.v_off[v] > hub_threshold) {
            int idx = atomicAdd(s.hub_count, 1);
            s.hubs[idx] = (int32_t)v;
        }
    }
}

// Piece offsets of the hubs (one workgroup): hub_piece_off[h] = number of
// kHubPiece pieces of hubs 0..h-1.
__global__ void __launch_bounds__(kBlock) k_hub_pieces(Graph g, State s) {
    __shared__ int wave_tmp[kWaves];
    __shared__ int carry;
    const int nh = *s.hub_count;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int h0 = 0; h0 < nh; h0 += kBlock) {
        const int h = h0 + threadIdx.x;
        int np = 0;
        if (h < nh) {
            const int v = s.hubs[h];
            np = (g.v_off[v + 1] - g.v_off[v] + kHubPiece - 1) / kHubPiece;
        }
        int total;
        int ex = block_exclusive_sum(np, wave_tmp, &total);
        if (h < nh) s.hub_piece_off[h] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) s.hub_piece_off[nh] = carry;
}

__global__ void __launch_bounds__(kBlock) k_zero_words(uint32_t *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

}  // namespace

hipError_t launch_init(const Launch &L, const Graph &g, uint32_t seed, const State &s,
                       uint32_t *bits, int crew) {
    hipLaunchKernelGGL(k_init, dim3(L.grid), dim3(kBlock), 0, L.stream, g, seed, s, bits, crew);
    return hipGetLastError();
}

hipError_t launch_validate(const Launch &L, const Graph &g, const State &s, int check_dual) {
    if (check_dual)
        hipLaunchKernelGGL(k_zero_words, dim3(L.grid), dim3(kBlock), 0, L.stream, s.vbits,
                           (g.kappa + 31) / 32);
    hipLaunchKernelGGL(k_validate, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s, check_dual);
    return hipGetLastError();
}

hipError_t launch_scatter(const Launch &L, const Graph &g, const State &s, int round) {
    (void)round;
    hipLaunchKernelGGL(k_scatter0, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s);
    return hipGetLastError();
}

hipError_t launch_retire(const Launch &L, const Graph &g, const State &s, int round, int scatter) {
    hipLaunchKernelGGL(k_retire, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s, round, scatter);
    return hipGetLastError();
}

hipError_t launch_vertex_max(const Launch &L, const Graph &g, const State &s, int round,
                             int hub_threshold) {
    if (round == 0) {
        hipLaunchKernelGGL(k_find_hubs, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s,
                           hub_threshold);
        hipLaunchKernelGGL(k_hub_pieces, dim3(1), dim3(kBlock), 0, L.stream, g, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_vertex_max, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s, round,
                       hub_threshold);
    return hipGetLastError();
}

hipError_t launch_test(const Launch &L, const Graph &g, const State &s, int round, int clear_next,
                       uint32_t *bits) {
    hipLaunchKernelGGL(k_test, dim3(L.grid), dim3(kBlock), 0, L.stream, g, s, round, clear_next,
                       bits);
    return hipGetLastError();
}

}  // namespace hgm
