// Schedule defaults: the values an hgm_opts schedule field of 0 stands for.
// Shared by the host driver (api.hip), which applies them, and the
// autotuner (tune.cpp), which starts its search from them.  Any value gives
// the same matching; these are the fastest measured on the MI355X.
#pragma once

#include <stdint.h>

namespace hgm {

constexpr int kDefaultHubThreshold = 8192;
constexpr int kBlocksPerCu = 8;
// Workgroups of the edge kernels (fixed, device independent, so that the
// workspace size does not depend on the device).  Swept on the MI355X (256
// CUs): one instance runs fastest at 1536 (power-law 1.030 -> 0.945 ms
// against 2048, hub-stress 1.287 -> 1.253, graphs 3-4% faster), a batch's
// round kernels at 4096 (18.3 -> 16.9 ms on 4,096 instances).
constexpr int kEdgeGrid = 1536;
constexpr int kEdgeGridBatch = 4096;
// The test clears the whole next maximum buffer by streaming when a round has
// at least n / kFullClearRatio live pins, else at each pin it visits.
constexpr int kFullClearRatio = 8;
constexpr int kHotDegree = 64;        // AUTO's round-0 form: degree of a hot vertex
constexpr int kFirstBatchPct = 40;    // first batch of rounds: 0.40 log2(kappa)
constexpr int kFirstBatchPctGraph = 35;
// Batches: instances with at most this many pins are matched whole by one
// workgroup each (k_solo) unless the options say otherwise: the batch's
// total pins / kSoloAutoDivisor, clamped to [kSoloAutoMin, kSoloAutoMax].
// One compute unit matches a solo instance at about 1.2e8 pins/s, the round
// kernels the whole batch at about 3e10, so this keeps the longest solo
// instance within about a quarter of the round kernels' time for the batch.
// Measured: 4,096 instances (4.8e8 pins) 16.35 -> 15.85 ms against the
// former fixed 2^20; 1,024 instances (1.2e8 pins) 8.4 -> about 5 ms.
constexpr int64_t kSoloAutoDivisor = 1024;
constexpr int64_t kSoloAutoMin = (int64_t)1 << 12;
constexpr int64_t kSoloAutoMax = (int64_t)1 << 20;
inline int64_t solo_auto_bound(int64_t kappa_total) {
    const int64_t b = kappa_total / kSoloAutoDivisor;
    return b < kSoloAutoMin ? kSoloAutoMin : b > kSoloAutoMax ? kSoloAutoMax : b;
}
// One instance: the tail workgroup takes over a round with at most this many
// live pins (and at most 65536 live edges).  Off unless asked for: on the
// synthetic workloads a round in one workgroup costs as much as a round of
// the grid-wide kernels (both are a chain of dependent memory accesses).
constexpr int kDefaultTailPins = -1;
// Binned maximum: automatic by default (0): on for large instances whose
// round 0 takes the vertex form, where it won (hub-stress 1.26 -> 1.18 ms);
// skewed degrees keep the atomic scatter, which won there (power-law 1.05
// against 1.11 ms with bins).
constexpr int kDefaultBinShift = 0;

}  // namespace hgm
