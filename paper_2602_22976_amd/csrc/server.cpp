// Request server (include/hgm.h, hgm_server_*): admits matching requests of
// mixed sizes against an HBM budget, keeps each admitted request's CSR and
// state resident in the caller's device arena until it is done, and batches
// requests as they arrive.
//
// Workers (threads, each with its own HIP stream) take turns forming a wave:
// every queued request that fits the free arena memory, up to max_batch, in
// arrival order.  A wave is uploaded into one arena block and matched with
// hgm_match_batch on the worker's stream; while it runs, the next worker
// forms the next wave from requests that arrived meanwhile, so waves overlap
// on the device.  Memory returns to the arena when a wave's results are
// copied out, which admits waiting requests.  A request's result does not
// depend on the wave it ran in (instances of a batch are independent).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "hgm.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) of the arena, 256-byte granularity.
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) {
        if (size_ > 0) free_[0] = size_;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    size_t size_;
    size_t used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Pending {
    hgm_request req;
    double t_submit;
};

// Byte layout of one wave inside its arena block.
struct WaveLayout {
    size_t v_base, e_base, pin_base, word_base, seeds, e_off, e_pins, v_off, v_edges, w, bits, ws,
        ws_bytes, total;
};

}  // namespace

struct hgm_server {
    char *arena_base;
    Arena arena;
    hgm_server_opts opts;
    int device;
    std::mutex mu;
    std::condition_variable cv_work;     // queue or memory changed
    std::condition_variable cv_results;  // results appended
    std::deque<Pending> queue;
    std::deque<hgm_result> results;
    bool stopping = false;
    bool forming = false;  // one worker at a time forms a wave, in arrival order
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;  // one per worker
    int64_t submitted = 0, completed = 0;
    int64_t stalls = 0;  // waits for arena memory with requests queued
    double stall_s = 0;

    hgm_server(char *base, size_t bytes) : arena_base(base), arena(bytes) {}
};

namespace {

// Sizes of a wave holding the given totals; the workspace is sized by
// hgm_batch_workspace_size on a descriptor with those totals.
WaveLayout wave_layout(int count, int64_t n, int64_t m, int64_t kappa, int64_t words,
                       const hgm_server_opts &o) {
    const bool vside = !o.edge_side_only;
    WaveLayout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t p = at;
        at = align256(at + std::max<size_t>(bytes, 1));
        return p;
    };
    L.v_base = take(8 * (size_t)(count + 1));
    L.e_base = take(8 * (size_t)(count + 1));
    L.pin_base = take(8 * (size_t)(count + 1));
    L.word_base = take(8 * (size_t)(count + 1));
    L.seeds = take(4 * (size_t)count);
    L.e_off = take(4 * (size_t)(m + count));
    L.e_pins = take(4 * (size_t)kappa);
    L.v_off = take(vside ? 4 * (size_t)(n + count) : 0);
    L.v_edges = take(vside ? 4 * (size_t)kappa : 0);
    L.w = take(4 * (size_t)m);
    L.bits = take(4 * (size_t)words);
    hgm_batch d;
    memset(&d, 0, sizeof(d));
    d.count = count;
    d.n_total = n;
    d.m_total = m;
    d.kappa_total = kappa;
    d.words_total = words;
    // Non-NULL placeholders: only sizes and the presence of the vertex side matter.
    d.v_base = d.e_base = d.pin_base = d.word_base = (const int64_t *)(uintptr_t)256;
    d.e_off = d.e_pins = (const int32_t *)(uintptr_t)256;
    if (vside) d.v_off = d.v_edges = (const int32_t *)(uintptr_t)256;
    d.w = d.seeds = (const uint32_t *)(uintptr_t)256;
    L.ws_bytes = hgm_batch_workspace_size(&d, &o.match);
    L.ws = take(L.ws_bytes);
    L.total = at;
    return L;
}

size_t words_of(int32_t m) { return ((size_t)m + 31) / 32; }

// off[0] = 0, off[i] <= off[i + 1], off[count] = total.  The loop keeps no
// early exit so that the compiler vectorises it.
bool offsets_ok(const int32_t *off, int64_t count, int64_t total) {
    if (off[0] != 0 || (int64_t)off[count] != total) return false;
    int bad = 0;
    for (int64_t i = 0; i < count; ++i) bad |= off[i + 1] < off[i];
    return bad == 0;
}

// Every id in [0, limit).
bool ids_ok(const int32_t *ids, int64_t len, int32_t limit) {
    uint32_t bad = 0;
    for (int64_t i = 0; i < len; ++i) bad |= (uint32_t)ids[i] >= (uint32_t)limit;
    return bad == 0;
}

// Size and NULL checks of a request (O(1)).
int request_args(const hgm_request &q, bool vside) {
    if (q.n < 0 || q.m < 0 || q.kappa < 0 || q.kappa >= ((int64_t)1 << 31)) return HGM_E_ARG;
    if ((q.m > 0 && (!q.e_off || !q.w || !q.bits_out)) || (q.kappa > 0 && !q.e_pins))
        return HGM_E_ARG;
    if (q.kappa > 0 && q.m == 0) return HGM_E_ARG;
    if (vside && (!q.v_off || (q.kappa > 0 && (!q.v_edges || q.n == 0)))) return HGM_E_ARG;
    return HGM_OK;
}

// O(kappa) content check (see hgm_request_check).
int request_content(const hgm_request &q, bool vside) {
    if (q.m > 0 && (!offsets_ok(q.e_off, q.m, q.kappa) || !ids_ok(q.e_pins, q.kappa, q.n)))
        return HGM_E_CSR;
    if (vside && (!offsets_ok(q.v_off, q.n, q.kappa) || !ids_ok(q.v_edges, q.kappa, q.m)))
        return HGM_E_CSR;
    return HGM_OK;
}

// A wave is one hgm_match_batch call, whose totals of vertices, edges, pins
// and bitmap bits are 32-bit.
constexpr int64_t kWaveLimit = ((int64_t)1 << 31) - 1;
// Default solo bound of a wave (measured on the served workload: 2^17 and
// below served 16% more requests per second than a bound of 2^20,
// with half the p99 latency).
constexpr int32_t kWaveSoloMaxKappa = 1 << 17;

void finish(hgm_server *S, const std::vector<Pending> &wave, int status, double t_admit) {
    const double t = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < wave.size(); ++i) {
        hgm_result r;
        memset(&r, 0, sizeof(r));
        r.id = wave[i].req.id;
        r.status = status;
        r.t_submit = wave[i].t_submit;
        r.t_admit = t_admit;
        r.t_done = t;
        r.wave_size = (int32_t)wave.size();
        S->results.push_back(r);
        S->completed += 1;
    }
    S->cv_results.notify_all();
}

int run_wave(hgm_server *S, hipStream_t stream, const std::vector<Pending> &wave, size_t off,
             const WaveLayout &L, int64_t n, int64_t m, int64_t kappa, int64_t words) {
    char *blk = S->arena_base + off;
    const int count = (int)wave.size();
    const bool vside = !S->opts.edge_side_only;
    std::vector<int64_t> vb(count + 1), eb(count + 1), pb(count + 1), wb(count + 1);
    std::vector<uint32_t> seeds(count);
    vb[0] = eb[0] = pb[0] = wb[0] = 0;
    for (int i = 0; i < count; ++i) {
        const hgm_request &q = wave[i].req;
        vb[i + 1] = vb[i] + q.n;
        eb[i + 1] = eb[i] + q.m;
        pb[i + 1] = pb[i] + q.kappa;
        wb[i + 1] = wb[i] + (int64_t)words_of(q.m);
        seeds[i] = q.seed;
    }
    // On failure, wait for the copies already queued (they read host vectors
    // local to this function) before returning.
#define SRV_TRY(x)                                       \
    do {                                                 \
        if ((x) != hipSuccess) {                         \
            (void)hipStreamSynchronize(stream);          \
            return HGM_E_HIP;                            \
        }                                                \
    } while (0)
    SRV_TRY(hipMemcpyAsync(blk + L.v_base, vb.data(), 8 * (count + 1), hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(blk + L.e_base, eb.data(), 8 * (count + 1), hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(blk + L.pin_base, pb.data(), 8 * (count + 1), hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(blk + L.word_base, wb.data(), 8 * (count + 1), hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(blk + L.seeds, seeds.data(), 4 * count, hipMemcpyHostToDevice, stream));
    for (int i = 0; i < count; ++i) {
        const hgm_request &q = wave[i].req;
        if (q.m > 0) {
            SRV_TRY(hipMemcpyAsync(blk + L.e_off + 4 * (eb[i] + i), q.e_off, 4 * ((size_t)q.m + 1),
                                   hipMemcpyHostToDevice, stream));
            SRV_TRY(hipMemcpyAsync(blk + L.w + 4 * eb[i], q.w, 4 * (size_t)q.m,
                                   hipMemcpyHostToDevice, stream));
        } else {
            static const int32_t zero = 0;
            SRV_TRY(hipMemcpyAsync(blk + L.e_off + 4 * (eb[i] + i), &zero, 4,
                                   hipMemcpyHostToDevice, stream));
        }
        if (q.kappa > 0) {
            SRV_TRY(hipMemcpyAsync(blk + L.e_pins + 4 * pb[i], q.e_pins, 4 * (size_t)q.kappa,
                                   hipMemcpyHostToDevice, stream));
            if (vside)
                SRV_TRY(hipMemcpyAsync(blk + L.v_edges + 4 * pb[i], q.v_edges,
                                       4 * (size_t)q.kappa, hipMemcpyHostToDevice, stream));
        }
        if (vside)
            SRV_TRY(hipMemcpyAsync(blk + L.v_off + 4 * (vb[i] + i), q.v_off, 4 * ((size_t)q.n + 1),
                                   hipMemcpyHostToDevice, stream));
    }
    hgm_batch d;
    memset(&d, 0, sizeof(d));
    d.count = count;
    d.n_total = n;
    d.m_total = m;
    d.kappa_total = kappa;
    d.words_total = words;
    d.v_base = (const int64_t *)(blk + L.v_base);
    d.e_base = (const int64_t *)(blk + L.e_base);
    d.pin_base = (const int64_t *)(blk + L.pin_base);
    d.word_base = (const int64_t *)(blk + L.word_base);
    d.seeds = (const uint32_t *)(blk + L.seeds);
    d.e_off = (const int32_t *)(blk + L.e_off);
    d.e_pins = (const int32_t *)(blk + L.e_pins);
    d.v_off = vside ? (const int32_t *)(blk + L.v_off) : nullptr;
    d.v_edges = vside ? (const int32_t *)(blk + L.v_edges) : nullptr;
    d.w = (const uint32_t *)(blk + L.w);
    int rc = hgm_match_batch(&d, (uint32_t *)(blk + L.bits), blk + L.ws, L.ws_bytes,
                             &S->opts.match, stream, nullptr);
    if (rc != HGM_OK) {
        (void)hipStreamSynchronize(stream);
        return rc;
    }
    for (int i = 0; i < count; ++i) {
        const hgm_request &q = wave[i].req;
        const size_t nw = words_of(q.m);
        if (nw && q.bits_out)
            SRV_TRY(hipMemcpyAsync(q.bits_out, blk + L.bits + 4 * wb[i], 4 * nw,
                                   hipMemcpyDeviceToHost, stream));
    }
    SRV_TRY(hipStreamSynchronize(stream));
#undef SRV_TRY
    return HGM_OK;
}

void worker_main(hgm_server *S, hipStream_t stream) {
    (void)hipSetDevice(S->device);  // checked by hgm_server_create on this device
    const int max_batch = S->opts.max_batch;
    for (;;) {
        std::vector<Pending> wave;
        size_t off = 0;
        WaveLayout L;
        int64_t n = 0, m = 0, kappa = 0, words = 0;
        double t_admit = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // Wait for our turn to form a wave and for a request to serve.
            S->cv_work.wait(lk, [&] { return S->stopping || (!S->forming && !S->queue.empty()); });
            if (S->queue.empty() && S->stopping) break;
            S->forming = true;
            for (;;) {
                // Grow the wave in arrival order while it fits the free memory.
                wave.clear();
                n = m = kappa = words = 0;
                bool fits_alone = true;
                size_t best = 0;
                for (size_t i = 0; i < S->queue.size() && (int)wave.size() < max_batch; ++i) {
                    const hgm_request &q = S->queue[i].req;
                    if (n + q.n > kWaveLimit || m + q.m > kWaveLimit ||
                        kappa + q.kappa > kWaveLimit ||
                        32 * (words + (int64_t)words_of(q.m)) > kWaveLimit)
                        break;  // submit checked that each request fits alone
                    const WaveLayout T = wave_layout((int)wave.size() + 1, n + q.n, m + q.m,
                                                     kappa + q.kappa,
                                                     words + (int64_t)words_of(q.m), S->opts);
                    size_t probe;
                    if (!S->arena.alloc(T.total, &probe)) {
                        if (wave.empty() && T.total > S->arena.size()) fits_alone = false;
                        break;
                    }
                    S->arena.release(probe, T.total);
                    wave.push_back(S->queue[i]);
                    n += q.n;
                    m += q.m;
                    kappa += q.kappa;
                    words += (int64_t)words_of(q.m);
                    best = T.total;
                }
                if (!fits_alone) {  // larger than the whole budget: fail it
                    Pending p = S->queue.front();
                    S->queue.pop_front();
                    lk.unlock();
                    finish(S, {p}, HGM_E_SIZE, now_s());
                    lk.lock();
                    if (S->queue.empty()) break;
                    continue;
                }
                if (!wave.empty()) {
                    L = wave_layout((int)wave.size(), n, m, kappa, words, S->opts);
                    (void)best;
                    if (S->arena.alloc(L.total, &off)) break;
                }
                // Nothing fits now: wait for memory to come back.
                const double w0 = now_s();
                S->cv_work.wait(lk);
                S->stalls += 1;
                S->stall_s += now_s() - w0;
                if (S->stopping && S->queue.empty()) break;
            }
            if (wave.empty()) {
                S->forming = false;
                S->cv_work.notify_all();
                if (S->stopping && S->queue.empty()) break;
                continue;
            }
            for (size_t i = 0; i < wave.size(); ++i) S->queue.pop_front();
            S->forming = false;
            t_admit = now_s();
        }
        S->cv_work.notify_all();  // the next worker may form the next wave now
        // Content check of every request before its arrays are uploaded: a
        // malformed request completes with HGM_E_CSR and never joins the
        // wave, so no kernel reads ids outside its own request.  The rest
        // run in a layout recomputed for them, which is no larger than the
        // block reserved for the whole wave.
        std::vector<Pending> good, bad;
        for (const Pending &p : wave)
            (request_content(p.req, !S->opts.edge_side_only) == HGM_OK ? good : bad).push_back(p);
        if (!bad.empty()) finish(S, bad, HGM_E_CSR, t_admit);
        int rc = HGM_OK;
        if (!good.empty()) {
            if (!bad.empty()) {
                n = m = kappa = words = 0;
                for (const Pending &p : good) {
                    n += p.req.n;
                    m += p.req.m;
                    kappa += p.req.kappa;
                    words += (int64_t)words_of(p.req.m);
                }
            }
            const WaveLayout G =
                bad.empty() ? L : wave_layout((int)good.size(), n, m, kappa, words, S->opts);
            rc = G.total <= L.total ? run_wave(S, stream, good, off, G, n, m, kappa, words)
                                    : HGM_E_SIZE;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(off, L.total);
        }
        S->cv_work.notify_all();
        if (!good.empty()) finish(S, good, rc, t_admit);
    }
}

}  // namespace

extern "C" {

int hgm_server_create(void *arena, size_t arena_bytes, const hgm_server_opts *opts,
                      hgm_server **out) {
    if (!out || !arena || arena_bytes == 0 || ((uintptr_t)arena & 255)) return HGM_E_ARG;
    hgm_server_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.workers < 0 || o.max_batch < 0 || o.workers > 64) return HGM_E_ARG;
    if (o.match.validate) return HGM_E_ARG;
    // Waves hold few requests (about one at the served workload's rate), so a
    // large request in the one-workgroup solo part would run on one compute
    // unit while the rest of the GPU idles: waves keep the solo part to
    // requests of at most kWaveSoloMaxKappa pins unless the options say.
    if (o.match.solo_max_kappa == 0) o.match.solo_max_kappa = kWaveSoloMaxKappa;
    if (o.edge_side_only != 0 && o.edge_side_only != 1) return HGM_E_ARG;
    // Without the vertex side only the edge-centric rounds can run.
    if (o.edge_side_only && o.match.variant == HGM_VARIANT_CREW) return HGM_E_ARG;
    if (o.workers == 0) o.workers = 2;
    if (o.max_batch == 0) o.max_batch = 1024;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HGM_E_HIP;
    // The workers' streams, created here so that a failure is reported.
    std::vector<hipStream_t> streams(o.workers, nullptr);
    for (int i = 0; i < o.workers; ++i) {
        if (hipStreamCreate(&streams[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipStreamDestroy(streams[j]);
            return HGM_E_HIP;
        }
    }
    hgm_server *S = new hgm_server((char *)arena, arena_bytes);
    S->opts = o;
    S->device = dev;
    S->streams = streams;
    for (int i = 0; i < o.workers; ++i) S->workers.emplace_back(worker_main, S, streams[i]);
    *out = S;
    return HGM_OK;
}

int hgm_server_submit(hgm_server *S, const hgm_request *req) {
    if (!S || !req) return HGM_E_ARG;
    const hgm_request &q = *req;
    // A bitmap larger than any wave can hold is a size error whatever else
    // the request carries.
    if (q.m > 0 && 32 * (int64_t)words_of(q.m) > kWaveLimit) return HGM_E_SIZE;
    const int rc = request_args(q, !S->opts.edge_side_only);
    if (rc != HGM_OK) return rc;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return HGM_E_ARG;
    S->queue.push_back(Pending{q, now_s()});
    S->submitted += 1;
    S->cv_work.notify_all();
    return HGM_OK;
}

int hgm_server_poll(hgm_server *S, hgm_result *out, int cap, double timeout_s) {
    if (!S || (cap > 0 && !out) || cap < 0) return HGM_E_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->results.empty() && timeout_s > 0)
        S->cv_results.wait_for(lk, std::chrono::duration<double>(timeout_s),
                               [&] { return !S->results.empty(); });
    int k = 0;
    while (k < cap && !S->results.empty()) {
        out[k++] = S->results.front();
        S->results.pop_front();
    }
    return k;
}

int hgm_server_info(hgm_server *S, hgm_server_state *st) {
    if (!S || !st) return HGM_E_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    st->queued = (int64_t)S->queue.size();
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->arena_bytes = S->arena.size();
    st->arena_used = S->arena.used();
    st->arena_peak = S->arena.peak();
    st->stalls = S->stalls;
    st->stall_s = S->stall_s;
    return HGM_OK;
}

int hgm_request_check(const hgm_request *req, int32_t vertex_side) {
    if (!req || (vertex_side != 0 && vertex_side != 1)) return HGM_E_ARG;
    const int rc = request_args(*req, vertex_side != 0);
    if (rc != HGM_OK) return rc;
    return request_content(*req, vertex_side != 0);
}

int hgm_server_destroy(hgm_server *S) {
    if (!S) return HGM_E_ARG;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    delete S;
    return HGM_OK;
}

}  // extern "C"
