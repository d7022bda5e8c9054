/* Multicore CPU local-max matching: a CPU baseline, not part of the library.
 *
 * The same iterated local-max rounds as the GPU path (Section 4.1,
 * Algorithm 1, concurrent-write form), parallelised over edges with OpenMP:
 * the paper's own CPU implementation of the method is a shared-memory
 * parallel version of these rounds (Section 6).  It is timed beside the GPU
 * path as a multicore comparison; the library never calls it.
 *
 * Key of edge e in round r: w(e) << 32 | H(s_r, e), with H the 32-bit
 * MurmurHash3 of e's four little-endian bytes (Appleby), s_r = seed for the
 * fixed order or H(seed, r) when the order is redrawn every round.
 *
 * Each round: (1) every live edge raises best[v] at its pins with an atomic
 * compare-and-swap maximum; (2) an edge equal to best[v] at all its pins is
 * matched, its pins marked done, and best[] is reset at the pins it read;
 * (3) live edges with a done pin are dropped and the rest compacted in order
 * (per-thread counts and a prefix sum).  Returns 0, or -1 on bad arguments
 * or allocation failure.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint32_t rotl(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

static inline uint32_t murmur4(uint32_t seed, uint32_t id) {
    uint32_t k = id * 0xcc9e2d51u;
    k = rotl(k, 15) * 0x1b873593u;
    uint32_t h = rotl(seed ^ k, 13) * 5u + 0xe6546b64u;
    h ^= 4u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    return h ^ (h >> 16);
}

static inline void atomic_max(uint64_t *p, uint64_t v) {
    uint64_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (cur < v &&
           !__atomic_compare_exchange_n(p, &cur, v, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
}

int cpu_local_max(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins,
                  const uint32_t *w, uint32_t seed, int reseed, int threads, uint32_t *bits,
                  int32_t *rounds_out, int64_t *sum_live_pins) {
    if (n < 0 || m < 0 || (m > 0 && (!e_off || !w || !bits))) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    uint64_t *best = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *live = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    uint8_t *keep = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    int nt = omp_get_max_threads();
    int64_t *tcount = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    if (!best || !done || !live || !next || !keep || !tcount) {
        free(best); free(done); free(live); free(next); free(keep); free(tcount);
        return -1;
    }
    memset(bits, 0, sizeof(uint32_t) * (size_t)((m + 31) / 32));
    for (int32_t e = 0; e < m; ++e) live[e] = e;
    int64_t n_live = m, pins_total = 0;
    int32_t round = 0;
    int used = 1;  /* threads of the compaction region */
    while (n_live > 0) {
        const uint32_t s = reseed ? murmur4(seed, (uint32_t)round) : seed;
        int64_t kap = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : kap)
        for (int64_t i = 0; i < n_live; ++i) {
            const int32_t e = live[i];
            const uint64_t k = ((uint64_t)w[e] << 32) | murmur4(s, (uint32_t)e);
            kap += e_off[e + 1] - e_off[e];
            for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) atomic_max(&best[e_pins[p]], k);
        }
        pins_total += kap;
        /* test; matched edges mark their pins and set their bit */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n_live; ++i) {
            const int32_t e = live[i];
            const uint64_t k = ((uint64_t)w[e] << 32) | murmur4(s, (uint32_t)e);
            int ok = 1;
            for (int32_t p = e_off[e]; p < e_off[e + 1] && ok; ++p)
                ok = __atomic_load_n(&best[e_pins[p]], __ATOMIC_RELAXED) == k;
            keep[i] = (uint8_t)ok;
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n_live; ++i) {
            const int32_t e = live[i];
            if (keep[i]) {
                __atomic_fetch_or(&bits[e >> 5], 1u << (e & 31), __ATOMIC_RELAXED);
                for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) done[e_pins[p]] = 1;
            }
        }
        /* reset best at every pin read this round (the survivors' pins are
         * among them), then retire and compact */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n_live; ++i) {
            const int32_t e = live[i];
            int alive = e_off[e + 1] > e_off[e];
            for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) {
                best[e_pins[p]] = 0;
                if (done[e_pins[p]]) alive = 0;
            }
            keep[i] = (uint8_t)alive;
        }
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num(), T = omp_get_num_threads();
#pragma omp single
            used = T;
            const int64_t lo = n_live * t / T, hi = n_live * (t + 1) / T;
            int64_t c = 0;
            for (int64_t i = lo; i < hi; ++i) c += keep[i];
            tcount[t + 1] = c;
#pragma omp barrier
#pragma omp single
            for (int u = 0; u < T; ++u) tcount[u + 1] += tcount[u];
            int64_t at = tcount[t];
            for (int64_t i = lo; i < hi; ++i)
                if (keep[i]) next[at++] = live[i];
        }
        n_live = tcount[used];
        int32_t *tmp = live;
        live = next;
        next = tmp;
        memset(tcount, 0, sizeof(int64_t) * ((size_t)nt + 1));
        round += 1;
    }
    if (rounds_out) *rounds_out = round;
    if (sum_live_pins) *sum_live_pins = pins_total;
    free(best); free(done); free(live); free(next); free(keep); free(tcount);
    return 0;
}
