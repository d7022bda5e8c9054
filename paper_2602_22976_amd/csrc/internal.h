// Internal interface between the round kernels (kernels.hip) and the host
// driver (api.hip).  Not installed; the public interface is include/hgm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hgm {

constexpr int kBlock = 256;  // threads per workgroup = edges (or vertices) per chunk

// Per-round counters, kept in a small device ring indexed by round % ring size.
struct RoundSlot {
    int32_t live;     // live edges at the start of the round (|L_r|)
    int32_t pad;
    int64_t kappa;    // sum of their sizes (kappa_r)
    int64_t matched;  // edges matched in the round
    uint64_t weight;  // their total weight
};

struct Graph {
    int32_t n, m;
    int64_t kappa;
    const int32_t *e_off;
    const int32_t *e_pins;
    const int32_t *v_off;
    const int32_t *v_edges;
    const uint32_t *w;
};

// Device state of one hgm_match call, carved out of the caller's workspace.
struct State {
    uint64_t *key;      // [m] packed key w<<32 | H(seed, e)
    uint64_t *best[2];  // [n] per-vertex maximum live key, double-buffered by round parity
    uint8_t *done;      // [n] vertex is a pin of a matched edge
    int32_t *list[2];   // [m] compacted live-edge lists, by round parity
    RoundSlot *slots;   // [ring]
    int32_t ring;
    int32_t *err;       // [1] validation error flag
    // CREW (vertex-centric) extras
    uint64_t *live_key; // [m] key while live, 0 once matched or retired
    int32_t *hubs;      // [n] vertices whose max is split over workgroups
    int32_t *hub_count; // [1]
    int32_t *hub_piece_off; // [n+1] piece offsets of the hubs
    uint32_t *vbits;    // [ceil(kappa/32)] validation: edge-side incidences seen
};

struct Launch {
    int grid;            // persistent workgroup count
    hipStream_t stream;
};

hipError_t launch_init(const Launch &L, const Graph &g, uint32_t seed, const State &s,
                       uint32_t *bits, int crew);
hipError_t launch_validate(const Launch &L, const Graph &g, const State &s, int check_dual);
hipError_t launch_scatter(const Launch &L, const Graph &g, const State &s, int round);
hipError_t launch_retire(const Launch &L, const Graph &g, const State &s, int round, int scatter);
hipError_t launch_vertex_max(const Launch &L, const Graph &g, const State &s, int round,
                             int hub_threshold);
hipError_t launch_test(const Launch &L, const Graph &g, const State &s, int round, int clear_next,
                       uint32_t *bits);

}  // namespace hgm
