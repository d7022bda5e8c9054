/*
 * hgm: weighted hypergraph matching by iterated local maxima on AMD MI355X.
 *
 * The method (paper: "Efficient Parallel Algorithms for Hypergraph Matching",
 * Section 4.1 Sequential Algorithm, Algorithms 1 and 2) works in rounds.
 * Every live hyperedge e carries a key; every vertex takes the largest key
 * over its live incident edges; an edge whose key is that largest value at
 * all of its pins joins the matching; every live edge that touches a pin of a
 * newly matched edge is retired (soft delete).  Rounds repeat until no live
 * edge remains.
 *
 * Key.  The paper perturbs the weights with random noise (Section 5.1, noise
 * in (0,1) for integer weights, extra noise for ties).  Here every edge gets
 * one fixed key for all rounds, compared as the tuple
 *     (w(e), H(seed, e), e)      larger is better,
 * where H(seed, e) = MurmurHash3_x86_32 of e's four little-endian bytes with
 * the given seed.  H is a bijection of e for a fixed seed, so keys are
 * distinct and the id never decides.  With a fixed strict order the local-max
 * rounds select exactly the matching that sequential greedy selects in that
 * order, so there is one correct output per (instance, seed).  opts->reseed
 * instead draws the tie-breaking priority afresh every round.
 *
 * Conventions for every entry point:
 *  - All array pointers inside hgm_csr, the output bitmap and the workspace
 *    are DEVICE pointers owned by the caller; the library allocates nothing.
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *    it in batches of rounds (opts->rounds_per_sync rounds, or a number the
 *    library predicts from the instance when that is 0); the stream is
 *    synchronised after each batch to test for termination, and the call
 *    returns when the matching is complete in device memory.
 *  - Return value: HGM_OK (0) or a negative HGM_E_* code; no exception or
 *    abort crosses this interface.  hgm_strerror() describes a code.
 *  - Calls that share a workspace must not overlap.
 */
#ifndef HGM_H
#define HGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HGM_OK 0
#define HGM_E_ARG (-1)         /* NULL pointer with a non-zero size, negative size, bad option */
#define HGM_E_CSR (-2)         /* malformed input detected by opts->validate (or by
                                  the binned maximum, see bin_shift) */
#define HGM_E_SIZE (-3)        /* kappa >= 2^31, or workspace too small */
#define HGM_E_ROUND_LIMIT (-4) /* opts->max_rounds rounds ran and live edges remain */
#define HGM_E_HIP (-5)         /* a HIP runtime call failed */

/* Round variants.  Both compute the same result (Algorithm 1 vs Algorithm 2
 * of the paper differ in how the per-vertex maximum is formed). */
#define HGM_VARIANT_AUTO 0 /* library choice per round */
#define HGM_VARIANT_CRCW 1 /* edge-centric: 64-bit atomic max of the key at each pin */
#define HGM_VARIANT_CREW 2 /* vertex-centric: segmented max over each vertex's edge list */

/* Hypergraph in the dual compressed form of the paper (Section 5.1):
 *   e_off   int32[m+1]  e_off[0] = 0, non-decreasing, e_off[m] = kappa
 *   e_pins  int32[kappa] pins of edge e are e_pins[e_off[e] .. e_off[e+1]),
 *                        distinct, each in [0, n)
 *   v_off   int32[n+1]  v_off[0] = 0, non-decreasing, v_off[n] = kappa
 *   v_edges int32[kappa] edges containing v are v_edges[v_off[v] .. v_off[v+1]);
 *                        the exact transpose of e_pins (any order inside a list)
 *   w       uint32[m]   edge weights (0 allowed)
 * Empty edges (size 0) are allowed and are matched (they conflict with
 * nothing); degree-0 vertices are allowed.  v_off/v_edges are required by
 * the CREW variant and by validation; AUTO uses them when given (round-0
 * form, hub pieces) and runs the edge-centric form without them; CRCW never
 * reads them.  Both may then be NULL. */
typedef struct hgm_csr {
    int32_t n, m;
    int64_t kappa;
    const int32_t *e_off;
    const int32_t *e_pins;
    const int32_t *v_off;
    const int32_t *v_edges;
    const uint32_t *w;
} hgm_csr;

/* Options; a NULL pointer means all defaults (the value 0 of each field). */
typedef struct hgm_opts {
    int32_t variant;         /* HGM_VARIANT_*; 0 = AUTO */
    int32_t hub_threshold;   /* vertices of larger degree are hubs: the
                                vertex-centric passes split their lists over
                                several workgroups, and AUTO's round-0 edge
                                scatter reduces their pins per workgroup in
                                LDS; 0 = library default (8192) */
    int32_t rounds_per_sync; /* rounds enqueued between host termination checks;
                                0 = library default */
    int32_t validate;        /* 1 = check the input first (extra O(kappa d) work
                                and one synchronisation); HGM_E_CSR on failure */
    int32_t max_rounds;      /* > 0: fail with HGM_E_ROUND_LIMIT if live edges
                                remain after this many rounds; 0 = no limit */
    int32_t reseed;          /* 0: one order for the whole run, priorities
                                H(seed, e).  1: priorities drawn afresh every
                                round, H(H(seed, r), e) in round r, weight still
                                first (the per-round random weights of
                                Algorithm 1, first phase).  The result is then
                                a maximal matching but in general not the
                                greedy one, and still exactly one bitmap per
                                (instance, seed).  Every variant; in
                                hgm_match_batch instance i uses
                                H(H(seed_i, r), local id). */
    int32_t pairs;           /* 1: a graph (every edge has exactly two pins,
                                Section 6.3): the pins of edge e are
                                e_pins[2e] and e_pins[2e + 1], e_off is not
                                read (may be NULL), kappa must be 2 m and
                                e_pins 8-byte aligned (else HGM_E_ARG).  Each
                                edge is then handled by one lane with one
                                8-byte pin load.  Not with HGM_VARIANT_CREW
                                nor with hgm_match_batch (HGM_E_ARG). */
    int32_t solo_max_kappa;  /* hgm_match_batch: instances with at most this
                                many pins (and at most 8 LDS tiles of
                                vertices, see hgm_solo_lds_vertices) are
                                matched whole by one workgroup each, every
                                round inside it, with their per-vertex state
                                in LDS; the others go through the round
                                kernels together.  0 = library default
                                (the batch's kappa_total / 1024, clamped to
                                [2^12, 2^20]), -1 = none. */
    /* Schedule (any value gives the same result; hgm_tune picks them per
     * shape).  0 = library default for each. */
    int32_t edge_grid;       /* workgroups of the edge-centric kernels, each
                                owning a fixed range of edge ids (default
                                1536 for one instance, 4096 for a batch; at
                                most 65536) */
    int32_t blocks_per_cu;   /* workgroups per compute unit of the vertex-
                                centric and setup kernels (default 8, at
                                most 32) */
    int32_t clear_ratio;     /* the test clears the next round's maximum by
                                one streaming pass when the round has at
                                least n / clear_ratio live pins, else at each
                                pin it visits (default 8) */
    int32_t hot_degree;      /* AUTO's round 0 is edge-centric when at least
                                half the pins lie on vertices of at least
                                this degree (default 64) */
    int32_t first_batch_pct; /* rounds enqueued before the first termination
                                check: pct / 100 * log2(kappa) (default 40,
                                35 for graphs; at most 400) */
    int32_t tail_pins;       /* hgm_match: once a round has at most this many
                                live pins (and at most 65536 live edges), one
                                workgroup runs every remaining round
                                (0 = library default: never; -1 = never) */
    int32_t bin_shift;       /* hgm_match, AUTO with the vertex side, offset
                                layout: the next round's per-vertex maximum
                                by propagation blocking instead of atomics,
                                in rounds with at least n / 2 surviving pins:
                                the retire pass writes each surviving pin's
                                (vertex, key) record to the bin of its
                                2^bin_shift-vertex range (hub pins excepted)
                                and one workgroup per bin reduces it in LDS.
                                It pays where most pins lie on low-degree
                                vertices.  0 = library default (automatic:
                                for n >= 2^17 and kappa >= 2^20, about 128
                                bins, used when the degree profile sends
                                round 0 to the vertex form, i.e. fewer than
                                half the pins lie on vertices of hot_degree
                                or more); 10..14 = that shift in every such
                                round; -1 = off.  At most 1024 bins, else
                                off.  Bins take 10 kappa bytes more
                                workspace.  Their capacities are v_off's
                                degree sums, so a v_off that is not e_pins'
                                transpose can overflow one: HGM_E_CSR. */
} hgm_opts;

/* Kernel classes reported by the timing statistics. */
#define HGM_K_SETUP 0      /* state clearing, batch keys, validation, hub pieces */
#define HGM_K_SCATTER 1    /* round-0 edge-centric maximum (CRCW) */
#define HGM_K_VERTEX_MAX 2 /* vertex-centric maximum (CREW) */
#define HGM_K_TEST 3       /* local-max test and marking */
#define HGM_K_RETIRE 4     /* retire + live-list compaction (+ next maximum in CRCW) */
#define HGM_K_SOLO 5       /* batches: every round of the instances matched by one workgroup */
#define HGM_K_TAIL 6       /* one instance: the remaining rounds run by one workgroup */
#define HGM_K_CLASSES 7

/* Optional statistics (host memory).  The arrays may be NULL; when given they
 * hold `cap` entries and receive, for round r < cap: the number of live edges
 * at the start of round r, the sum of their sizes (live pin incidences), the
 * number of edges matched in round r and the sum of their sizes.  `rounds`
 * is the number of rounds run, `matched` = |M|, `weight` = w(M) (64-bit sum).
 * Timing (input field `timing` = 1): every kernel is bracketed by HIP events
 * on the call's stream; kernel_ms / kernel_launches receive the summed device
 * time and launch count per HGM_K_* class over the rounds that had live
 * edges, and round_ms (if non-NULL) the device time of each round's kernels
 * (its maximum, test, and the retire pass that ends it). */
typedef struct hgm_stats {
    int32_t rounds;
    int64_t matched;
    uint64_t weight;
    int64_t *live_edges;
    int64_t *live_pins;
    int64_t *matched_per_round;
    int64_t *matched_pins;
    int32_t cap;
    int32_t timing;
    float *round_ms;
    double kernel_ms[HGM_K_CLASSES];
    int32_t kernel_launches[HGM_K_CLASSES];
} hgm_stats;

/* Bytes of device workspace hgm_match needs for this instance and options.
 * Returns 0 when g is NULL or its sizes are invalid. */
size_t hgm_workspace_size(const hgm_csr *g, const hgm_opts *opts);

/* Match one hypergraph.
 *   g             input (device arrays, see hgm_csr)
 *   seed          seed of the priority hash H
 *   matched_bits  device uint32[ceil(m/32)], written: bit (e % 32) of word
 *                 e / 32 is 1 iff edge e is in the matching (LSB first)
 *   workspace     device memory of at least hgm_workspace_size() bytes,
 *                 256-byte aligned; contents on entry are ignored
 *   opts, stream  see above; stats may be NULL
 * Paper: Algorithm 1 (CRCW) and Algorithm 2 (CREW), with the soft delete of
 * Section 4.1 realised as a compacted list of live edges. */
int hgm_match(const hgm_csr *g, uint32_t seed, uint32_t *matched_bits, void *workspace,
              size_t ws_bytes, const hgm_opts *opts, void *stream, hgm_stats *stats);

/* hgm_match without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a fixed array of
 * hgm_noalloc_max_bytes() bytes (64 MiB) in the library's own device memory,
 * one per GPU, held from the library's load until the process ends; its
 * address is looked up on the first call on each device.  The entry point
 * calls no hipMalloc / hipFree or other allocating routine.
 *   Arguments, results and errors as hgm_match, plus: HGM_E_SIZE when the
 * instance needs more workspace than the array holds (hgm_workspace_size()
 * > hgm_noalloc_max_bytes()); HGM_E_ARG for stats->timing = 1 (timing
 * creates HIP events).  Every call on one GPU uses that GPU's one array and
 * leaves its contents behind (the next call clears what it needs), so calls
 * that overlap on one GPU -- on different streams or threads -- race and
 * must be serialised by the caller. */
int hgm_match_noalloc(const hgm_csr *g, uint32_t seed, uint32_t *matched_bits,
                      const hgm_opts *opts, void *stream, hgm_stats *stats);
/* Size in bytes of hgm_match_noalloc's per-GPU workspace array. */
size_t hgm_noalloc_max_bytes(void);

/* A batch of independent hypergraphs matched in one call.  Instances keep
 * their own (local) ids, so instance i's slices are byte-identical to its
 * standalone hgm_csr; all arrays are the instances' arrays concatenated in
 * order.  Base arrays have count + 1 entries (prefix sums, [0] = 0):
 *   v_base[i]    first vertex of instance i   (v_base[count] = n_total)
 *   e_base[i]    first edge                   (e_base[count] = m_total)
 *   pin_base[i]  first incidence              (pin_base[count] = kappa_total)
 *   word_base[i] first bitmap word            (word_base[count] = words_total)
 *   e_off        int32[m_total + count]: instance i's m_i + 1 local offsets
 *                start at e_off[e_base[i] + i]
 *   e_pins       int32[kappa_total] local vertex ids
 *   v_off        int32[n_total + count]: instance i's n_i + 1 local offsets
 *                start at v_off[v_base[i] + i] (may be NULL, as in hgm_csr)
 *   v_edges      int32[kappa_total] local edge ids (may be NULL)
 *   w            uint32[m_total]
 *   seeds        uint32[count] priority-hash seed of each instance
 * All pointers are device pointers.  Instance i's matching is written to
 * words word_base[i] .. word_base[i] + ceil(m_i / 32) of the output bitmap
 * (edge e at bit e % 32 of word word_base[i] + e / 32) and equals what
 * hgm_match returns for that instance and seed alone.  Limits: n_total,
 * m_total, kappa_total and 32 * words_total below 2^31. */
typedef struct hgm_batch {
    int32_t count;
    int64_t n_total, m_total, kappa_total, words_total;
    const int64_t *v_base;
    const int64_t *e_base;
    const int64_t *pin_base;
    const int64_t *word_base;
    const int32_t *e_off;
    const int32_t *e_pins;
    const int32_t *v_off;
    const int32_t *v_edges;
    const uint32_t *w;
    const uint32_t *seeds;
} hgm_batch;

/* Vertices of one LDS tile of the one-workgroup path on the current device:
 * an instance of a batch with at most this many vertices forms each round's
 * maximum in one pass; one with up to 8 tiles' worth in one pass per tile;
 * larger ones go through the round kernels. */
int hgm_solo_lds_vertices(void);

/* Workspace bytes for hgm_match_batch (0 on invalid sizes or options). */
size_t hgm_batch_workspace_size(const hgm_batch *b, const hgm_opts *opts);

/* Match every instance of a batch in one pass of launches: the instances are
 * vertex-disjoint, so the local-max rounds of their union select each
 * instance's own matching; each instance leaves the live set when its last
 * live edge is gone, and the call ends when all have.  Options and stats as
 * for hgm_match (stats aggregate over the batch); opts->validate is not
 * supported here (HGM_E_ARG): validate instances with hgm_match. */
int hgm_match_batch(const hgm_batch *b, uint32_t *matched_bits, void *workspace, size_t ws_bytes,
                    const hgm_opts *opts, void *stream, hgm_stats *stats);

/* ---------------------------------------------------------------------------
 * Schedule autotuner.  The schedule fields of hgm_opts (edge_grid,
 * blocks_per_cu, hub_threshold, hot_degree, clear_ratio, first_batch_pct,
 * and solo_max_kappa for batches) change how the work is laid out, never the
 * result.  hgm_tune times whole matchings of the given instance (median of
 * `reps` calls after one untimed call) under candidate schedules, by
 * coordinate descent from `base` (NULL or 0 fields: the defaults), checks
 * that every candidate produces the starting schedule's bitmap, and returns
 * the fastest schedule in *best (base's other fields kept).  With a cache
 * path (or, when `cache` is NULL, the HGM_TUNE_CACHE environment variable)
 * the result is also stored in that text file under a key of the device
 * (architecture and compute units) and the shape bucket (kind, variant,
 * layout, per-round priorities, round(log2 kappa), mean edge size, and for
 * batches round(log2 count)); hgm_tuned_opts reads it back for an instance
 * of the same bucket.  The workspace must hold hgm_tune_workspace_size()
 * bytes (the largest candidate edge grid); matched_bits receives the
 * matching.  Not part of the paper: a schedule search of this library. */
typedef struct hgm_tune_report {
    double ms_default;       /* median time of the starting schedule */
    double ms_best;          /* median time of the schedule returned */
    int32_t evaluations;     /* schedules timed */
    int32_t identical;       /* 1: every candidate gave the starting bitmap */
} hgm_tune_report;

size_t hgm_tune_workspace_size(const hgm_csr *g, const hgm_opts *base);
size_t hgm_tune_batch_workspace_size(const hgm_batch *b, const hgm_opts *base);
int hgm_tune(const hgm_csr *g, uint32_t seed, uint32_t *matched_bits, void *workspace,
             size_t ws_bytes, const hgm_opts *base, void *stream, int32_t reps,
             const char *cache, hgm_opts *best, hgm_tune_report *report);
int hgm_tune_batch(const hgm_batch *b, uint32_t *matched_bits, void *workspace, size_t ws_bytes,
                   const hgm_opts *base, void *stream, int32_t reps, const char *cache,
                   hgm_opts *best, hgm_tune_report *report);
/* Looks up the cached schedule for this instance's bucket (variant, pairs
 * and reseed taken from *opts) and writes its fields into *opts: HGM_OK, or
 * HGM_E_ARG when there is no cache or no entry (opts unchanged). */
int hgm_tuned_opts(const char *cache, const hgm_csr *g, hgm_opts *opts);
int hgm_tuned_batch_opts(const char *cache, const hgm_batch *b, hgm_opts *opts);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of matching requests on one GPU.
 *
 * The caller gives the server a device arena (its HBM budget).  Requests
 * (host arrays) are queued by hgm_server_submit.  Worker threads, each with
 * its own HIP stream, take turns forming a wave from every queued request
 * that fits the arena's free memory (arrival order, at most max_batch),
 * upload it into one arena block, match it with hgm_match_batch and copy each
 * request's bitmap back; requests arriving meanwhile go into the next wave,
 * which another worker runs concurrently.  A wave's memory returns to the
 * arena when it completes, admitting waiting requests.  A request's bitmap is
 * exactly hgm_match's for that instance and seed, whatever it ran with.  A
 * request larger than the whole arena completes with status HGM_E_SIZE.  A
 * wave also stays within hgm_match_batch's 32-bit totals (n, m, kappa and
 * 32 * bitmap words below 2^31). */
typedef struct hgm_request {
    int64_t id;              /* caller's tag, echoed in the result */
    int32_t n, m;
    int64_t kappa;
    const int32_t *e_off;    /* HOST arrays in the hgm_csr layout (the vertex */
    const int32_t *e_pins;   /* side is required unless edge_side_only); they */
    const int32_t *v_off;    /* must stay valid until the request's result has */
    const int32_t *v_edges;  /* been polled.  Pinned host memory makes the */
                             /* uploads asynchronous. */
    const uint32_t *w;
    uint32_t seed;
    uint32_t *bits_out;      /* HOST, ceil(m/32) words, written before the result is posted */
} hgm_request;

typedef struct hgm_result {
    int64_t id;
    int32_t status;          /* HGM_OK or an HGM_E_* code */
    int32_t wave_size;       /* requests matched together with this one */
    double t_submit;         /* steady-clock seconds: submitted, admitted into a */
    double t_admit;          /* wave (memory reserved), bitmap copied back */
    double t_done;
} hgm_result;

typedef struct hgm_server_opts {
    int32_t workers;         /* concurrent waves (threads and streams); 0 = 2 */
    int32_t max_batch;       /* requests per wave at most; 0 = 1024 */
    hgm_opts match;          /* options of every wave's matching (validate unsupported;
                                solo_max_kappa 0 means 2^17 here: a wave holds few
                                requests, and a large one is faster in the round
                                kernels than on one compute unit) */
    int32_t edge_side_only;  /* 1: requests carry only the edge side (v_off and v_edges
                                are ignored and may be NULL); half the bytes to upload,
                                and every round is edge-centric (with CREW: HGM_E_ARG) */
} hgm_server_opts;

typedef struct hgm_server_state {
    int64_t queued, submitted, completed;
    uint64_t arena_bytes, arena_used, arena_peak;  /* peak never exceeds arena_bytes */
    int64_t stalls;          /* times a worker found requests queued but none fitting the
                                free arena memory, and waited for memory to return */
    double stall_s;          /* total time spent in those waits */
} hgm_server_state;

typedef struct hgm_server hgm_server;

/* arena: device memory, 256-byte aligned, owned by the caller and unused by
 * it until hgm_server_destroy returns.  The current device is the server's.
 * HGM_E_HIP when the workers' streams cannot be created. */
int hgm_server_create(void *arena, size_t arena_bytes, const hgm_server_opts *opts,
                      hgm_server **out);
/* Queues a request (non-blocking, thread-safe).  HGM_E_SIZE when its bitmap
 * alone exceeds a wave's limit (m > 2^31 - 32; checked first); else
 * HGM_E_ARG for negative sizes, kappa >= 2^31, kappa > 0 with m = 0, or a
 * NULL array that its sizes require.  Before its arrays are uploaded, a worker checks the
 * request's content as hgm_request_check does; a malformed request then
 * completes with status HGM_E_CSR and never joins a wave, so no kernel of
 * the wave reads an id outside that request's own arrays. */
int hgm_server_submit(hgm_server *server, const hgm_request *req);

/* Host-side O(kappa) check of a request's arrays (no GPU needed): e_off
 * starts at 0, never decreases and ends at kappa; every pin lies in [0, n);
 * with vertex_side = 1 the same for v_off (ending at kappa) and incident
 * edge ids in [0, m).  HGM_OK, HGM_E_ARG (sizes or NULL arrays, as
 * hgm_server_submit) or HGM_E_CSR.  Repeated pins inside an edge and whether
 * the vertex side is exactly the transpose are not checked (opts->validate
 * of hgm_match checks both); they cannot make a kernel touch memory outside
 * the request's own arrays, and only change that request's own result. */
int hgm_request_check(const hgm_request *req, int32_t vertex_side);
/* Moves up to `cap` finished results to `out`, waiting up to timeout_s
 * seconds for the first; returns how many were written (or an HGM_E_* code). */
int hgm_server_poll(hgm_server *server, hgm_result *out, int cap, double timeout_s);
int hgm_server_info(hgm_server *server, hgm_server_state *state);
/* Finishes every queued request, stops the workers and frees the server. */
int hgm_server_destroy(hgm_server *server);

/* Short English description of an HGM_* code (static storage). */
const char *hgm_strerror(int code);

/* Library version as major*10000 + minor*100 + patch. */
int hgm_version(void);

/* Digest of the sources and compiler flags the library was built from
 * (static storage), so that a binding can refuse a stale build. */
const char *hgm_source_digest(void);

#ifdef __cplusplus
}
#endif

#endif /* HGM_H */
