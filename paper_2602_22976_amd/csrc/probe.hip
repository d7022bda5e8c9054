// Memory-system ceilings of the access patterns the round kernels use,
// measured on the device (built into libhgm_probe.so, driven by
// bench.py --ceilings; not part of the matching library):
//   stream      coalesced 16-byte loads over a buffer (the HBM streaming rate)
//   gather8     8-byte loads at random indices into a buffer of a given size
//               (best[] reads of the test and the filtered scatter)
//   gather1     1-byte loads at random indices (done[] reads of the retire)
//   atomic8     device-scope 64-bit atomic max at random indices (the scatter's
//               atomics), fire-and-forget
//   filtered8   a gather, then the atomic only where the value rises (the
//               scatter as the kernels run it)
//   hot8        64-bit atomic max on one address (a hub's best entry)
//   launches    back-to-back launches of an empty kernel of the round kernels'
//               shape, on a stream and replayed from a captured HIP graph
//   scatter     the per-vertex maximum of a list of (vertex, key) records,
//               best[v] = max key of v's records, in two forms on the same
//               records: filtered device atomics (the round kernels' form, on a
//               cleared best[]) and propagation blocking (records binned by
//               vertex range, each range max-reduced in LDS and written whole)
// Indices come from a caller buffer of random uint32 values reduced modulo
// the element count inside the kernel, read coalesced.  Every kernel folds
// what it loads into one word per thread so that no load is dead code.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) k_stream(const uint4 *p, int64_t n, uint32_t *sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc ^= a.x ^ b.y ^ c.z ^ d.w;
    }
    for (; i < n; i += stride) acc ^= p[i].x;
    if (acc == 0x9e3779b9u) sink[0] = acc;  // practically never: keeps the loads live
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_gather(const T *p, uint32_t elems,
                                                     const uint32_t *idx, int64_t count,
                                                     uint32_t *sink) {
    uint64_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + 3 * stride < count; i += 4 * stride) {
        const uint32_t a = idx[i] % elems, b = idx[i + stride] % elems,
                       c = idx[i + 2 * stride] % elems, d = idx[i + 3 * stride] % elems;
        acc += (uint64_t)p[a] + (uint64_t)p[b] + (uint64_t)p[c] + (uint64_t)p[d];
    }
    for (; i < count; i += stride) acc += (uint64_t)p[idx[i] % elems];
    if (acc == 0x9e3779b97f4a7c15ull) sink[0] = (uint32_t)acc;
}

__global__ void __launch_bounds__(kThreads) k_atomic(uint64_t *p, uint32_t elems,
                                                     const uint32_t *idx, int64_t count,
                                                     int filtered) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
        const uint32_t h = idx[i];
        const uint32_t at = h % elems;
        const uint64_t v = ((uint64_t)(h >> 12) << 32) | h;  // random key
        if (filtered) {
            const uint64_t cur =
                __hip_atomic_load(&p[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur >= v) continue;
        }
        __hip_atomic_fetch_max(&p[at], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// An almost empty kernel of the round kernels' shape: each workgroup reads
// one counter and returns (a late round's launch with nothing to do).
__global__ void __launch_bounds__(kThreads) k_empty(const int *cnt, int *sink) {
    if (cnt[blockIdx.x] == -1 && threadIdx.x == 0) sink[0] = 1;  // never: cnt holds zeros
}

// --- scatter forms --------------------------------------------------------

__global__ void __launch_bounds__(kThreads) k_fill0(uint64_t *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// One record per lane and step: a read of best[v] (workgroup scope, so it
// hits in L2; best only grows, so a stale value is a lower bound), then the
// device atomic only where the key raises it.
__global__ void __launch_bounds__(kThreads) k_scatter_atomic(const uint32_t *vid,
                                                             const uint64_t *key, int64_t count,
                                                             uint64_t *best) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
        const uint32_t v = vid[i];
        const uint64_t k = key[i];
        if (__hip_atomic_load(&best[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < k)
            __hip_atomic_fetch_max(&best[v], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

constexpr int kBinThreads = 1024;
constexpr int kMaxBins = 4096;
constexpr int kBinUnroll = 4;

// Propagation blocking, writing side.  Workgroup p takes a contiguous slice
// of the records, counts them per bin (vertex range of 2^rb ids) in LDS,
// reserves its run in each bin with one device atomic on the bin's cursor,
// and writes every record (local index, key) to its bin.  Bin j's records
// live at bin_base[j] + [0, cursor[j]); bin_base holds capacities that
// cannot be exceeded (every record of the bin).
__global__ void __launch_bounds__(kBinThreads) k_bin_write(const uint32_t *vid,
                                                           const uint64_t *key, int64_t count,
                                                           int rb, int nb,
                                                           const int64_t *bin_base,
                                                           uint32_t *cursor, uint16_t *bin_v,
                                                           uint64_t *bin_key) {
    __shared__ uint32_t cnt[kMaxBins];
    __shared__ unsigned long long pos[kMaxBins];
    const int64_t lo = count * blockIdx.x / gridDim.x;
    const int64_t hi = count * (blockIdx.x + 1) / gridDim.x;
    for (int j = threadIdx.x; j < nb; j += kBinThreads) cnt[j] = 0;
    __syncthreads();
    constexpr int64_t step = (int64_t)kBinThreads * kBinUnroll;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += step) {
        uint32_t v[kBinUnroll];
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBinThreads;
            v[u] = i < hi ? vid[i] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u)
            if (v[u] != 0xFFFFFFFFu) atomicAdd(&cnt[v[u] >> rb], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += kBinThreads) {
        const uint32_t c = cnt[j];
        pos[j] = c ? (unsigned long long)(bin_base[j] + atomicAdd(&cursor[j], c)) : 0ull;
    }
    __syncthreads();
    const uint32_t mask = (1u << rb) - 1u;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += step) {
        uint32_t v[kBinUnroll];
        uint64_t k[kBinUnroll];
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBinThreads;
            v[u] = i < hi ? vid[i] : 0xFFFFFFFFu;
            k[u] = i < hi ? key[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            if (v[u] == 0xFFFFFFFFu) continue;
            const unsigned long long at = atomicAdd(&pos[v[u] >> rb], 1ull);
            bin_v[at] = (uint16_t)(v[u] & mask);
            bin_key[at] = k[u];
        }
    }
}

// Propagation blocking, reducing side: workgroup j max-reduces bin j's
// records into an LDS tile of 2^rb keys, writes the tile to best[] whole
// (entries without records become 0, so best needs no clear) and resets the
// bin's cursor for the next pass.
__global__ void __launch_bounds__(kBinThreads) k_bin_reduce(const int64_t *bin_base,
                                                            uint32_t *cursor,
                                                            const uint16_t *bin_v,
                                                            const uint64_t *bin_key, int rb,
                                                            int64_t n, uint64_t *best) {
    extern __shared__ unsigned long long tile[];
    const int j = blockIdx.x;
    const int r = 1 << rb;
    for (int t = threadIdx.x; t < r; t += kBinThreads) tile[t] = 0;
    const int64_t b0 = bin_base[j];
    const int64_t c = cursor[j];
    __syncthreads();
    constexpr int64_t step = (int64_t)kBinThreads * kBinUnroll;
    for (int64_t i0 = threadIdx.x; i0 < c; i0 += step) {
        uint16_t v[kBinUnroll];
        uint64_t k[kBinUnroll];
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * kBinThreads;
            v[u] = i < c ? bin_v[b0 + i] : 0;
            k[u] = i < c ? bin_key[b0 + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u)
            if (k[u]) atomicMax(&tile[v[u]], (unsigned long long)k[u]);
    }
    __syncthreads();
    const int64_t v0 = (int64_t)j << rb;
    for (int t = threadIdx.x; t < r; t += kBinThreads)
        if (v0 + t < n) best[v0 + t] = tile[t];
    if (threadIdx.x == 0) cursor[j] = 0;
}

}  // namespace

extern "C" {

// Average microseconds per launch of `launches` back-to-back empty kernels
// of `grid` workgroups: plain stream launches (*stream_us) and the same
// sequence captured once in a HIP graph and replayed (*graph_us; capture
// and instantiation are not timed).  cnt: device int[grid] of zeros.
int hgm_probe_launches(const int *cnt, int *sink, int grid, int launches, int reps,
                       double *stream_us, double *graph_us) {
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) return -1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
    auto enqueue = [&]() {
        for (int i = 0; i < launches; ++i)
            hipLaunchKernelGGL(k_empty, dim3(grid), dim3(kThreads), 0, st, cnt, sink);
    };
    enqueue();  // warm up
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    float ms = 0.f, best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        hipEventRecord(a, st);
        enqueue();
        hipEventRecord(b, st);
        hipEventSynchronize(b);
        hipEventElapsedTime(&ms, a, b);
        best = ms < best ? ms : best;
    }
    *stream_us = 1e3 * best / launches;
    hipGraph_t g;
    hipGraphExec_t ge;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return -1;
    enqueue();
    if (hipStreamEndCapture(st, &g) != hipSuccess) return -1;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) return -1;
    hipGraphLaunch(ge, st);  // warm up
    hipStreamSynchronize(st);
    best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        hipEventRecord(a, st);
        hipGraphLaunch(ge, st);
        hipEventRecord(b, st);
        hipEventSynchronize(b);
        hipEventElapsedTime(&ms, a, b);
        best = ms < best ? ms : best;
    }
    *graph_us = 1e3 * best / launches;
    hipGraphExecDestroy(ge);
    hipGraphDestroy(g);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipStreamDestroy(st);
    return (int)hipGetLastError();
}

// Each launcher enqueues one probe on `stream` and returns the HIP status.
int hgm_probe_stream(const void *buf, int64_t bytes, uint32_t *sink, void *stream, int grid) {
    hipLaunchKernelGGL(k_stream, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream,
                       (const uint4 *)buf, bytes / 16, sink);
    return (int)hipGetLastError();
}

int hgm_probe_gather(const void *buf, int64_t bytes, int elem_bytes, const uint32_t *idx,
                     int64_t count, uint32_t *sink, void *stream, int grid) {
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather<uint64_t>, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream,
                           (const uint64_t *)buf, (uint32_t)(bytes / 8), idx, count, sink);
    else
        hipLaunchKernelGGL(k_gather<uint8_t>, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream,
                           (const uint8_t *)buf, (uint32_t)bytes, idx, count, sink);
    return (int)hipGetLastError();
}

// elems = 1 puts every atomic on one address.
int hgm_probe_atomic(void *buf, int64_t elems, const uint32_t *idx, int64_t count, int filtered,
                     void *stream, int grid) {
    hipLaunchKernelGGL(k_atomic, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream,
                       (uint64_t *)buf, (uint32_t)elems, idx, count, filtered);
    return (int)hipGetLastError();
}

// best[v] = max over the records (vid[i], key[i]) with vid[i] == v, by
// filtered device atomics; clear != 0 first zeroes best[0 .. n).
int hgm_probe_scatter_atomic(const uint32_t *vid, const uint64_t *key, int64_t count,
                             uint64_t *best, int64_t n, int clear, void *stream, int grid) {
    if (clear)
        hipLaunchKernelGGL(k_fill0, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, best, n);
    if (count > 0)
        hipLaunchKernelGGL(k_scatter_atomic, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream,
                           vid, key, count, best);
    return (int)hipGetLastError();
}

// The same maximum by propagation blocking: phase 1 writes the records to
// bins of 2^rb vertices (producers workgroups), phase 2 reduces each bin and
// writes best[0 .. n) whole.  bin_base: int64[nb + 1] with nb = ceil(n / 2^rb),
// bin j's capacity bin_base[j + 1] - bin_base[j] at least its record count;
// cursor: uint32[nb], zero on entry and left zero; bin_v / bin_key: at least
// bin_base[nb] entries.  Returns -1 for nb > 4096, rb outside [6, 14] or
// vertex ids of 2^32 - 1 (the empty-slot mark).
int hgm_probe_scatter_binned(const uint32_t *vid, const uint64_t *key, int64_t count,
                             uint64_t *best, int64_t n, int rb, const int64_t *bin_base,
                             uint32_t *cursor, uint16_t *bin_v, uint64_t *bin_key, int phases,
                             void *stream, int producers) {
    if (rb < 6 || rb > 14 || n <= 0 || n >= 0xFFFFFFFFll || producers <= 0) return -1;
    const int64_t nb = (n + (1ll << rb) - 1) >> rb;
    if (nb > kMaxBins) return -1;
    const size_t lds = (size_t)8 << rb;
    static size_t granted = 0;
    if (granted < lds) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bin_reduce),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return -1;
        granted = lds;
    }
    if ((phases & 1) && count > 0)
        hipLaunchKernelGGL(k_bin_write, dim3(producers), dim3(kBinThreads), 0, (hipStream_t)stream,
                           vid, key, count, rb, (int)nb, bin_base, cursor, bin_v, bin_key);
    if (phases & 2)
        hipLaunchKernelGGL(k_bin_reduce, dim3((unsigned)nb), dim3(kBinThreads), lds,
                           (hipStream_t)stream, bin_base, cursor, bin_v, bin_key, rb, n, best);
    return (int)hipGetLastError();
}

}  // extern "C"
