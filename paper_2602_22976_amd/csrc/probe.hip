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

}  // extern "C"
