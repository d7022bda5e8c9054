/*
 * Oracle for weighted hypergraph matching by iterated local maxima.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain CPU definition that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product library never
 * links or calls it, and it shares no code with the GPU kernels.
 *
 * Notation follows the paper (Preliminaries): n = |V|, m = |E|, |e| the size
 * of hyperedge e, kappa = sum of |e|.  The hypergraph is held in the dual
 * compressed form of the paper's implementation section (Sequential
 * Algorithm): e_off/e_pins list the pins of each edge, v_off/v_edges list the
 * edges incident to each vertex.
 *
 * Edge order.  The paper perturbs integer weights with small noise so that
 * all weights become distinct (Implementation, Sequential Algorithm) and
 * suggests edge ids as a strict order (Experiments on Graphs, Quality).  Here
 * the order is fixed once: edges are compared as the tuple
 *     (w(e), H(seed, e), e)
 * lexicographically, larger is better, where H is MurmurHash3_x86_32 of the
 * edge id's four little-endian bytes under the given seed.  The weight comes
 * first, so the order refines the weight order and the 1/d guarantee of
 * Lemma 1 applies unchanged.
 *
 * What is computed.
 *  - oracle_greedy: the sequential greedy 1/d approximation the paper uses as
 *    its single-core baseline (Introduction; Experiments on Hypergraphs): sort
 *    all edges by the order above, best first, and take an edge when none of
 *    its pins is taken yet.
 *  - oracle_local_max_reseed: the same rounds with fresh tie-breaking
 *    priorities every round (see local_max_impl).
 *  - oracle_local_max: the round-based local-max algorithm (Sequential
 *    Algorithm; Algorithm 2, CREW form) with the fixed order.  Each round every
 *    active vertex records its best active incident edge T[v]; an active edge e
 *    whose P_e = #{v in e : T[v] = e} equals |e| joins the matching; its pins
 *    become newly completed; every active edge containing a newly completed
 *    vertex becomes inactive; newly completed vertices become inactive.  It
 *    also reports, per round r, the number of active edges |L_r|, their pin
 *    count kappa_r and the number of edges matched in the round.
 * For a strict total order both produce the same matching; the tests check
 * that, and check each against properties fixed by the paper's lemmas.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_NOMEM (-2)
#define ORACLE_E_ROUNDS (-3)

/* ---------------------------------------------------------------------- */
/* MurmurHash3_x86_32 (Austin Appleby, public domain), written out from its
 * published definition: 4-byte little-endian blocks mixed with c1, c2 and
 * rotations, a tail of up to 3 bytes, length xor, then the fmix32 finaliser. */
static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t oracle_murmur3_x86_32(const uint8_t *data, uint64_t len, uint32_t seed) {
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h1 = seed;
    uint64_t nblocks = len / 4;
    for (uint64_t i = 0; i < nblocks; ++i) {
        uint32_t k1 = (uint32_t)data[4 * i] | ((uint32_t)data[4 * i + 1] << 8) |
                      ((uint32_t)data[4 * i + 2] << 16) | ((uint32_t)data[4 * i + 3] << 24);
        k1 *= c1;
        k1 = rotl32(k1, 15);
        k1 *= c2;
        h1 ^= k1;
        h1 = rotl32(h1, 13);
        h1 = h1 * 5u + 0xe6546b64u;
    }
    const uint8_t *tail = data + nblocks * 4;
    uint32_t k1 = 0;
    switch (len & 3) {
    case 3: k1 ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2: k1 ^= (uint32_t)tail[1] << 8;  /* fall through */
    case 1:
        k1 ^= tail[0];
        k1 *= c1;
        k1 = rotl32(k1, 15);
        k1 *= c2;
        h1 ^= k1;
    }
    h1 ^= (uint32_t)len;
    return fmix32(h1);
}

/* H(seed, e): the hash of edge id e's four little-endian bytes. */
static uint32_t priority(uint32_t seed, int32_t e) {
    uint32_t u = (uint32_t)e;
    uint8_t b[4] = {(uint8_t)u, (uint8_t)(u >> 8), (uint8_t)(u >> 16), (uint8_t)(u >> 24)};
    return oracle_murmur3_x86_32(b, 4, seed);
}

void oracle_priorities(uint32_t seed, int32_t m, uint32_t *out) {
    for (int32_t e = 0; e < m; ++e) out[e] = priority(seed, e);
}

/* Edge order as a tuple; returns >0 when a ranks above b. */
typedef struct { uint32_t w, h; int32_t e; } edge_rank;

static int rank_cmp(const edge_rank *a, const edge_rank *b) {
    if (a->w != b->w) return a->w > b->w ? 1 : -1;
    if (a->h != b->h) return a->h > b->h ? 1 : -1;
    if (a->e != b->e) return a->e > b->e ? 1 : -1;
    return 0;
}

static int rank_cmp_desc(const void *a, const void *b) {
    return -rank_cmp((const edge_rank *)a, (const edge_rank *)b);
}

static int check_edges(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins) {
    if (n < 0 || m < 0 || !e_off) return ORACLE_E_ARG;
    if (e_off[0] != 0) return ORACLE_E_ARG;
    for (int32_t e = 0; e < m; ++e)
        if (e_off[e + 1] < e_off[e]) return ORACLE_E_ARG;
    for (int64_t i = 0; i < e_off[m]; ++i)
        if (e_pins[i] < 0 || e_pins[i] >= n) return ORACLE_E_ARG;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Sequential greedy.  bits has ceil(m/32) words; edge e is bit (e % 32) of
 * word e / 32.  Returns the matched count and total weight. */
int oracle_greedy(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins,
                  const uint32_t *w, uint32_t seed, uint32_t *bits,
                  int64_t *matched_count, uint64_t *matched_weight) {
    int rc = check_edges(n, m, e_off, e_pins);
    if (rc) return rc;
    edge_rank *order = (edge_rank *)malloc(sizeof(edge_rank) * (size_t)(m > 0 ? m : 1));
    uint8_t *taken = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!order || !taken) { free(order); free(taken); return ORACLE_E_NOMEM; }
    for (int32_t e = 0; e < m; ++e) {
        order[e].w = w[e];
        order[e].h = priority(seed, e);
        order[e].e = e;
    }
    qsort(order, (size_t)m, sizeof(edge_rank), rank_cmp_desc);
    memset(bits, 0, sizeof(uint32_t) * (size_t)((m + 31) / 32));
    int64_t count = 0;
    uint64_t weight = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t e = order[i].e;
        int free_all = 1;
        for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p)
            if (taken[e_pins[p]]) { free_all = 0; break; }
        if (!free_all) continue;
        for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) taken[e_pins[p]] = 1;
        bits[e / 32] |= 1u << (e % 32);
        count += 1;
        weight += w[e];
    }
    free(order);
    free(taken);
    if (matched_count) *matched_count = count;
    if (matched_weight) *matched_weight = weight;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Seed of round r when the order is drawn afresh every round: the priority
 * hash of the round number under the call's seed, H(seed, r). */
static uint32_t round_seed(uint32_t seed, int32_t r) { return priority(seed, r); }

/* Round-based local max.  Per-round statistics are written for the first
 * `cap` rounds (arrays may be NULL when cap is 0).  max_rounds <= 0 means no
 * limit; otherwise exceeding it returns ORACLE_E_ROUNDS.  With reseed = 0 the
 * order is the fixed tuple (w, H(seed, e), e); with reseed = 1 round r ranks
 * edges by (w, H(H(seed, r), e), e): fresh tie-breaking priorities every
 * round, as the paper's per-round random weights (Algorithm 1, first phase),
 * with the weight still deciding first. */
static int local_max_impl(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins,
                          const int32_t *v_off, const int32_t *v_edges, const uint32_t *w,
                          uint32_t seed, int reseed, int32_t max_rounds, uint32_t *bits,
                          int32_t *rounds_out, int64_t *live_edges, int64_t *live_pins,
                          int64_t *matched_per_round, int32_t cap) {
    int rc = check_edges(n, m, e_off, e_pins);
    if (rc) return rc;
    if (!v_off || v_off[0] != 0 || v_off[n] != e_off[m]) return ORACLE_E_ARG;
    for (int32_t v = 0; v < n; ++v)
        if (v_off[v + 1] < v_off[v]) return ORACLE_E_ARG;
    for (int64_t i = 0; i < v_off[n]; ++i)
        if (v_edges[i] < 0 || v_edges[i] >= m) return ORACLE_E_ARG;

    edge_rank *rk = (edge_rank *)malloc(sizeof(edge_rank) * (size_t)(m > 0 ? m : 1));
    uint8_t *edge_active = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    uint8_t *edge_new = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    uint8_t *vert_active = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    uint8_t *vert_new = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int32_t *T = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!rk || !edge_active || !edge_new || !vert_active || !vert_new || !T) {
        rc = ORACLE_E_NOMEM;
        goto out;
    }
    for (int32_t e = 0; e < m; ++e) {
        rk[e].w = w[e];
        rk[e].h = priority(seed, e);
        rk[e].e = e;
        edge_active[e] = 1;
    }
    for (int32_t v = 0; v < n; ++v) vert_active[v] = 1;
    memset(bits, 0, sizeof(uint32_t) * (size_t)((m + 31) / 32));

    int32_t round = 0;
    for (;;) {
        int64_t n_live = 0, k_live = 0;
        for (int32_t e = 0; e < m; ++e)
            if (edge_active[e]) { n_live += 1; k_live += e_off[e + 1] - e_off[e]; }
        if (n_live == 0) break;
        if (max_rounds > 0 && round >= max_rounds) { rc = ORACLE_E_ROUNDS; break; }
        if (round < cap) { live_edges[round] = n_live; live_pins[round] = k_live; }
        if (reseed) {
            const uint32_t rs = round_seed(seed, round);
            for (int32_t e = 0; e < m; ++e) rk[e].h = priority(rs, e);
        }

        /* Every active vertex records its best active incident edge (-1: none). */
        for (int32_t v = 0; v < n; ++v) {
            T[v] = -1;
            if (!vert_active[v]) continue;
            for (int32_t i = v_off[v]; i < v_off[v + 1]; ++i) {
                int32_t e = v_edges[i];
                if (!edge_active[e]) continue;
                if (T[v] < 0 || rank_cmp(&rk[e], &rk[T[v]]) > 0) T[v] = e;
            }
        }
        /* An active edge that is the best at every pin joins the matching. */
        int64_t matched = 0;
        for (int32_t e = 0; e < m; ++e) {
            edge_new[e] = 0;
            if (!edge_active[e]) continue;
            int32_t P = 0;
            for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) P += (T[e_pins[p]] == e);
            if (P == e_off[e + 1] - e_off[e]) {
                bits[e / 32] |= 1u << (e % 32);
                edge_new[e] = 1;
                matched += 1;
            }
        }
        if (round < cap) matched_per_round[round] = matched;
        /* A vertex is newly completed when one of its edges was just matched. */
        for (int32_t v = 0; v < n; ++v) {
            vert_new[v] = 0;
            if (!vert_active[v]) continue;
            for (int32_t i = v_off[v]; i < v_off[v + 1]; ++i)
                if (edge_new[v_edges[i]]) vert_new[v] = 1;
        }
        /* Matched edges and every edge with a newly completed pin go inactive. */
        for (int32_t e = 0; e < m; ++e) {
            if (!edge_active[e]) continue;
            int any = edge_new[e];
            for (int32_t p = e_off[e]; p < e_off[e + 1]; ++p) any |= vert_new[e_pins[p]];
            if (any) edge_active[e] = 0;
        }
        for (int32_t v = 0; v < n; ++v)
            if (vert_new[v]) vert_active[v] = 0;
        round += 1;
    }
    if (rounds_out) *rounds_out = round;
out:
    free(rk);
    free(edge_active);
    free(edge_new);
    free(vert_active);
    free(vert_new);
    free(T);
    return rc;
}

int oracle_local_max(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins,
                     const int32_t *v_off, const int32_t *v_edges, const uint32_t *w,
                     uint32_t seed, int32_t max_rounds, uint32_t *bits, int32_t *rounds_out,
                     int64_t *live_edges, int64_t *live_pins, int64_t *matched_per_round,
                     int32_t cap) {
    return local_max_impl(n, m, e_off, e_pins, v_off, v_edges, w, seed, 0, max_rounds, bits,
                          rounds_out, live_edges, live_pins, matched_per_round, cap);
}

int oracle_local_max_reseed(int32_t n, int32_t m, const int32_t *e_off, const int32_t *e_pins,
                            const int32_t *v_off, const int32_t *v_edges, const uint32_t *w,
                            uint32_t seed, int32_t max_rounds, uint32_t *bits,
                            int32_t *rounds_out, int64_t *live_edges, int64_t *live_pins,
                            int64_t *matched_per_round, int32_t cap) {
    return local_max_impl(n, m, e_off, e_pins, v_off, v_edges, w, seed, 1, max_rounds, bits,
                          rounds_out, live_edges, live_pins, matched_per_round, cap);
}

/* Key H(H(seed, r), e) of the reseeded order, for tests. */
uint32_t oracle_round_priority(uint32_t seed, int32_t round, int32_t e) {
    return priority(round_seed(seed, round), e);
}

/* ---------------------------------------------------------------------- */
/* Exhaustive injectivity check of H(seed, .) over all 2^32 ids: marks every
 * hash value in a 512 MiB bitmap and returns how many values were hit twice
 * (0 for a bijection), or -2 when the bitmap cannot be allocated. */
int64_t oracle_priority_collisions(uint32_t seed) {
    uint64_t *seen = (uint64_t *)calloc((size_t)1 << 26, sizeof(uint64_t));
    if (!seen) return ORACLE_E_NOMEM;
    int64_t dup = 0;
    uint32_t x = 0;
    do {
        uint8_t b[4] = {(uint8_t)x, (uint8_t)(x >> 8), (uint8_t)(x >> 16), (uint8_t)(x >> 24)};
        uint32_t h = oracle_murmur3_x86_32(b, 4, seed);
        uint64_t bit = (uint64_t)1 << (h & 63);
        if (seen[h >> 6] & bit) dup += 1;
        seen[h >> 6] |= bit;
        x += 1;
    } while (x != 0);
    free(seen);
    return dup;
}
