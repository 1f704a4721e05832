/*
 * hbmax.h -- C ABI of the MI355X (gfx950) memory-efficient IMM hot path.
 *
 * The library samples random reverse-reachable (RR) sets on the transposed
 * graph under the IC or LT diffusion model, stores them plain, Huffman-coded
 * (a codebook learned from a warm-up block) or with hot vertices in bitmap
 * rows, and runs greedy max-coverage seed selection directly on that store.
 * The operations follow the paper's problem statement (Introduction and
 * Background: G = (V, E, w), a diffusion model and a budget k), the RR-set
 * definitions of the Background section, Alg. 1 (sampling-and-encoding),
 * Alg. 2 and Alg. 3 with Eq. 3 (selection on the coded sets) and Eq. 1
 * (the IMM sampling schedule of Tang et al.).
 *
 * Conventions shared by every call:
 *  - Every call returns an hbm_status; nothing else crosses the ABI on error,
 *    and host outputs are left untouched when the status is not HBM_OK.
 *    hbm_last_error() gives a human-readable reason for the last failure.
 *  - A context owns all device memory it allocates.  Device memory comes from
 *    the optional allocator callback, else hipMalloc.  Calls on one context
 *    are not thread-safe; distinct contexts are independent.
 *  - All work is issued on the stream given to hbm_create.  Calls that return
 *    host outputs synchronise that stream before returning.
 *  - Vertex ids are int32 in [0, n); edge counts are below 2^32; the number of
 *    RR sets held by a store is below 2^31.
 *  - RR set j under seed s is a pure function of (graph, model, s, j): the
 *    Philox4x32-10 stream is keyed by s and counted by (j, edge group or
 *    vertex, tag), so any prefix of a store equals the sets a larger request
 *    would produce, independent of launch shape or block size.
 */
#ifndef HBMAX_H
#define HBMAX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hbm_status {
    HBM_OK = 0,
    HBM_EINVAL = 1,  /* bad argument or malformed graph */
    HBM_ENOMEM = 2,  /* device allocation failed */
    HBM_EBUDGET = 3, /* the store went over its budget, or a final theta reached 2^31 sets */
    HBM_EDEVICE = 4, /* a HIP call failed */
    HBM_ESTATE = 5   /* call made in the wrong order (e.g. sampling before a graph) */
} hbm_status;

/* Diffusion models of the Background section. */
typedef enum hbm_model { HBM_IC = 0, HBM_LT = 1 } hbm_model;

/* Edge probabilities: EDGE uses the given weight w(u,v); WC (weighted cascade)
   uses 1/indeg(v), rounded to float32, and ignores w. */
typedef enum hbm_prob { HBM_PROB_EDGE = 0, HBM_PROB_WC = 1 } hbm_prob;

/* Store encodings (Alg. 1).  HUFFMAN: Huffmax byte strings with verbatim
   copies of codeless vertices.  HOT_BITMAP: the top fraction of vertices by
   warm-up frequency go to bitmap rows (Bitmax restricted to hot vertices),
   the rest are kept as plain ids.  HUFFMAN_HOT_BITMAP: hot rows plus Huffman
   coding of the remaining vertices.  BITMAX: the Bitmax encoding section's
   dense bit matrix, one row of ceil(theta / 64) words for every vertex (set j
   is bit j of each row; the padding bits stay zero), selection by Alg. 3.
   AUTO: Alg. 1's choice after characterizing the warm-up block with Eq. 2:
   BITMAX when the skewness is negative and the density is above 1/32 (the
   RRR-set characterization section's threshold), else HUFFMAN;
   hbm_store_stats.encoding reports the choice. */
typedef enum hbm_enc {
    HBM_ENC_NONE = 0,
    HBM_ENC_HUFFMAN = 1,
    HBM_ENC_HOT_BITMAP = 2,
    HBM_ENC_HUFFMAN_HOT_BITMAP = 3,
    HBM_ENC_BITMAX = 4,
    HBM_ENC_AUTO = 5
} hbm_enc;

typedef struct hbm_ctx hbm_ctx;

/* Device allocator callback (e.g. a framework's caching allocator).  alloc
   returns device memory or NULL; release frees it.  Both run on the calling
   thread.  Pass NULL to hbm_create to use hipMalloc / hipFree. */
typedef struct hbm_allocator {
    void *(*alloc)(size_t bytes, void *user);
    void (*release)(void *ptr, void *user);
    void *user;
} hbm_allocator;

/* Sizes of the current store.  Bytes counted per part; B/RR = store_bytes / nsets. */
typedef struct hbm_store_stats {
    int64_t nsets;          /* RR sets held (theta) */
    int64_t members;        /* total vertex occurrences */
    int64_t warmup_sets;    /* W: sets in the warm-up block */
    int32_t encoding;       /* hbm_enc in use (AUTO resolves to BITMAX or HUFFMAN once the warm-up is done) */
    int32_t nhot;           /* hot vertices with bitmap rows */
    int32_t alphabet;       /* vertices with a Huffman code */
    int32_t max_code_len;   /* longest code, bits */
    int32_t ustar_enc;      /* warm-up top coded vertex (-1 if none) */
    int32_t escape_bits;    /* width of a verbatim id */
    int64_t escapes;        /* codeless occurrences copied verbatim */
    uint64_t payload_bits;  /* Huffman stream bits */
    int64_t index_bytes;    /* per-set offsets (Huffman: + one code-boundary byte per 256 payload bits) */
    int64_t bitmap_bytes;   /* hot rows */
    int64_t raw_bytes;      /* plain ids (NONE / cold part of HOT_BITMAP) */
    int64_t codebook_bytes; /* lengths, packed per-vertex code table (8 B per vertex), symbol table, hot and array lists */
    int64_t store_bytes;    /* index + payload + bitmap + raw (codebook excluded) */
    double skewness;        /* Eq. 2 over the warm-up block */
    double density;         /* Eq. 2 over the warm-up block */
    int32_t narray;         /* hot vertices with array rows (hbm_set_row_containers) */
    int64_t array_entries;  /* 16-bit set offsets held by the array rows */
    int64_t array_bytes;    /* array rows: per-chunk offsets + entries (in store_bytes) */
} hbm_store_stats;

/* Result details of hbm_imm. */
typedef struct hbm_imm_stats {
    int32_t rounds;             /* estimation rounds run */
    int64_t theta_round[64];    /* theta_i per round */
    uint64_t cov_round[64];     /* coverage of the round's k seeds */
    double lb;                  /* lower bound of OPT (1 if no round passed) */
    int64_t theta_final;        /* ceil(lambda* / LB) */
    int64_t nsets_final;        /* sets in the final store: max(theta_final, last theta_i) */
    uint64_t coverage;          /* sets covered by the final seeds */
    double influence;           /* n * coverage / nsets_final */
    double lambda_prime, lambda_star;
    double t_sample_ms, t_encode_ms, t_select_ms, t_total_ms;  /* t_encode_ms: building the codebook and
                                                                  hot set from the warm-up block (host wall
                                                                  time, part of t_sample_ms) */
    hbm_store_stats store;
} hbm_imm_stats;

/* ---------------------------------------------------------------- lifetime */

/* Create a context on HIP device `device`, issuing work on `stream`
   (a hipStream_t; NULL = the null stream).  `alloc` may be NULL. */
hbm_status hbm_create(hbm_ctx **out, int device, void *stream, const hbm_allocator *alloc);

/* Free every device buffer owned by the context.  NULL is a no-op. */
void hbm_destroy(hbm_ctx *ctx);

/* Reason for the last non-OK status on this context ("" if none). */
const char *hbm_last_error(const hbm_ctx *ctx);

/* Cap, in bytes, on the RR store (index + payload + bitmap rows, as counted in
   hbm_store_stats.store_bytes; 0 = no cap).  Sampling stops with HBM_EBUDGET after
   the block that took the store over the cap (see hbm_sample_rr). */
hbm_status hbm_set_budget(hbm_ctx *ctx, int64_t store_bytes);

/* ---------------------------------------------------------------- graph */

/* Load G = (V, E, w) (the Influence Maximization Problem subsection of the
 * Background: a directed graph with edge weights, under the IC or LT model;
 * RR sets are walked on its transpose, as the RR-set definition of the RIS
 * subsection states) given as a FORWARD CSR in device memory:
 *   row_ptr  int64[n+1]  out-edge offsets, row_ptr[0] = 0, non-decreasing, row_ptr[n] = m
 *   dst      int32[m]    target of each out-edge
 *   w        float32[m]  weight of each out-edge, or NULL when prob == HBM_PROB_WC
 * The buffers are only read during the call.  The library builds the
 * transposed graph (in-edges of v ordered by ascending source; edge id =
 * position in that order), then the per-edge (IC-EDGE) or per-vertex (WC)
 * live thresholds, or for LT the running float32 sum of in-weights along each
 * in-row (added left to right).
 * HBM_EINVAL when: n <= 0, m < 0 or m >= 2^32, row_ptr malformed, a target
 * out of range, a self-loop, a duplicate (u,v), a weight that is NaN or
 * negative, an IC weight above 1, or an LT in-weight sum (float32, added
 * left to right) above 1 + 2^-20 + indeg(v) * 2^-23 (the second term covers
 * float32 accumulation of rows already normalised to sum 1).
 * Loading a graph resets the RR store. */
hbm_status hbm_load_graph(hbm_ctx *ctx, int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *dst,
                          const float *w, hbm_model model, hbm_prob prob);

/* ---------------------------------------------------------------- store */

/* Choose the store encoding.  warmup_frac: the warm-up block is the first
 * W = min(theta, max(1, ceil(warmup_frac * theta))) sets of the first
 * sampling request after a reset (Alg. 1's first block); the codebook and the
 * hot set come from its vertex frequencies and are never rebuilt.  hot_frac:
 * the hot set is the ceil(hot_frac * n) vertices with the highest warm-up
 * frequency (ties to the lower id; vertices never seen are excluded).
 * hot_frac is ignored by BITMAX and AUTO.
 * Resets the store.  HBM_EINVAL for fractions outside (0, 1] where used, and for
 * a Huffman encoding (or AUTO) on a graph of 2^27 or more vertices (the decode tables pack
 * a vertex id and a code length into 32 bits; hbm_load_graph refuses such a graph
 * while a Huffman encoding is set). */
hbm_status hbm_set_encoding(hbm_ctx *ctx, hbm_enc enc, double warmup_frac, double hot_frac);

/* Density gate of the hot set: a vertex qualifies only if it is in at least
 * max(1, ceil(min_density * W)) of the W warm-up sets.  A bitmap row costs one bit
 * per set and a stored id 32 bits per occurrence, so with min_density = 1/32 a
 * vertex gets a row only where the row is the smaller form (the density threshold
 * of the RRR-set characterization section, applied per vertex).  Default 0 (the
 * plain top-fraction rule).  Resets the store.  HBM_EINVAL outside [0, 1]. */
hbm_status hbm_set_hot_density(hbm_ctx *ctx, double min_density);

/* Implicit roots: every RR set holds its root, and root_j is a pure function of
 * (seed, j) (the first Philox draw of set j), so with on = 1 a store leaves the root
 * out of the set's plain ids or Huffman string and regenerates it wherever the set
 * is decoded, searched or decremented; a root with a bitmap row keeps its bit (and
 * a BITMAX store is unchanged).  Saves the root's cost in every set (4 bytes as a
 * plain id, its code or escape in a Huffman string); results are unchanged.
 * Default 0.  Resets the store.  HBM_EINVAL unless on is 0 or 1. */
hbm_status hbm_set_implicit_roots(hbm_ctx *ctx, int32_t on);

/* Row containers for the hot set (the Roaring-style bitmap compression that the
 * Huffman Coding and Bitmap Compression background section names): with on = 1, a hot
 * vertex found in fewer than W/16 of the W warm-up sets gets an ARRAY row instead of a
 * bitmap row.  The sets are cut into chunks of 2^16 consecutive sets; in each chunk an
 * array row holds the ascending 16-bit offsets (j mod 2^16) of the chunk's sets that
 * hold the vertex, 16 bits per occurrence against a bitmap row's one bit per set.
 * Layout (hbm_export HBM_A_ARR_*): rows in hot order (ARR_HOT); offsets chunk-major,
 * nar + 1 per chunk, into one entry array (ARR_OFF, ARR_LOW); row a of chunk c is
 * ARR_LOW[ARR_OFF[c (nar + 1) + a] .. ARR_OFF[c (nar + 1) + a + 1]).  Selection reads
 * an array row as the list of its sets (u* with an array row marks them; counts of
 * array rows drop by the entries of newly covered sets).  Affects HOT_BITMAP and
 * HUFFMAN_HOT_BITMAP only; results are unchanged.  Default 0.  Resets the store.
 * HBM_EINVAL unless on is 0 or 1. */
hbm_status hbm_set_row_containers(hbm_ctx *ctx, int32_t on);

/* Spill of plain ids to host memory (the equal-memory comparison of the
 * Evaluation section, where an uncompressed store that outgrows memory spills to
 * slower storage): with device_bytes > 0, a store that keeps plain ids (NONE, and
 * the cold part of HOT_BITMAP) holds at most floor(device_bytes / 16) * 4 of them in
 * device memory; the rest go to pinned host memory (hipHostMalloc, mapped and
 * coherent) that the sampling, selection and decode kernels read and write over
 * the bus.  Results are
 * unchanged; only where the ids live, and so the speed, differs.  0 (default) keeps
 * every id on the device.  Huffman and bitmap parts never spill.  Resets the store.
 * HBM_EINVAL for device_bytes < 0 or in [1, 15]. */
hbm_status hbm_set_spill(hbm_ctx *ctx, int64_t device_bytes);

/* RIS sampling (the RIS, IMM and Ripples subsection of the Background: each RR
 * set is the set of vertices that reach a uniformly random root over live edges)
 * followed by Alg. 1's encoding of every block (the first block is the warm-up
 * that fixes the codebook and hot set).
 * Make the store hold RR sets j = 0 .. theta-1 under `seed`.  Appends when the
 * seed matches and theta grows; a different seed, or a smaller theta, resets
 * the store first.  HBM_ESTATE without a graph; HBM_EINVAL if theta < 0 or
 * theta >= 2^31.  Sets are added in blocks; HBM_EBUDGET (the store went over
 * hbm_set_budget's limit) and HBM_ENOMEM leave a valid prefix of sets in the
 * store: those of the blocks completed up to and including the one that failed
 * the budget. */
hbm_status hbm_sample_rr(hbm_ctx *ctx, int64_t theta, uint64_t seed);

/* Greedy max coverage over the store (the Seed Selection paragraph; Alg. 2 /
 * Alg. 3 picking exactly k seeds): each pick is the unselected vertex in the
 * most uncovered sets, the lowest id winning ties.  Host outputs:
 *   seeds int32[k], gains uint64[k] (uncovered sets each pick covered),
 *   coverage = sum of gains.
 * The store is not modified.  HBM_EINVAL if k < 1 or k > n. */
hbm_status hbm_select_seeds(hbm_ctx *ctx, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage);

/* hbm_select_seeds for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results as hbm_select_seeds, bit for bit, but the selection state
 * (counts, covered and newly covered bits, argmax partials, seed keys, the queue of
 * long strings) lives in a fixed device array of 48 MiB that the library holds on
 * each device it runs on until the process ends; nothing is allocated, and the
 * call neither times nor profiles its kernels.  The state needs, each part rounded
 * up to 256 bytes: 4 n + n / 8 + 2 * 8 ceil(theta / 64) + 8 k + 8 * 8 * CUs, plus
 * 4 (theta + 2) for a Huffman store; a call that needs more returns HBM_EINVAL
 * (2^22 vertices with 2^22 sets fit under any encoding).  Counts are dense (one
 * per vertex) whatever HBM_TUNE_SPARSE_COUNTS says.  Every call on a device
 * shares that device's array, so calls that overlap on one device (two contexts on
 * different streams or threads) race and must be serialised by the caller; each
 * call clears what it needs at its start.  The store must have been sampled by
 * the calling context (hbm_sample_rr), whose allocations are its own. */
hbm_status hbm_select_seeds_noalloc(hbm_ctx *ctx, int32_t k, int32_t *seeds, uint64_t *gains, uint64_t *coverage);

/* Full IMM (Eq. 1 read as Tang et al.'s lambda'; their lower bound and final
 * theta): l is adjusted to l (1 + ln 2 / ln n); estimation round i samples
 * theta_i = ceil(lambda' / (n / 2^i)) sets and selects k seeds; the first
 * round with n cov_i / theta_i >= (1 + sqrt(2) eps) n / 2^i fixes
 * LB = n cov_i / (theta_i (1 + sqrt(2) eps)); then theta = ceil(lambda* / LB)
 * and the final k seeds come from max(theta, theta_last) sets.  RR sets are
 * reused across rounds.  The store is reset first.  Host outputs: seeds
 * int32[k], gains uint64[k] (may be NULL), stats (may be NULL). */
hbm_status hbm_imm(hbm_ctx *ctx, int32_t k, double eps, double l, uint64_t seed, int32_t *seeds, uint64_t *gains,
                   hbm_imm_stats *stats);

/* ---------------------------------------------------------------- batched instances */

/* One IMM query: k seeds at accuracy eps with failure exponent l (l = 1 gives
 * probability at least 1 - 1/n), RR sets drawn under Philox seed `seed`. */
typedef struct hbm_query {
    int32_t k;
    double eps;
    double l;
    uint64_t seed;
} hbm_query;

/* Full IMM (as hbm_imm) for `count` independent instances at once, each on its
 * own context with its own graph and encoding.  Every step of the method runs as
 * one grouped launch over all instances still in that step (sampling blocks,
 * encoding, each greedy iteration), so many small instances share launches
 * instead of paying for each.  Each instance's result equals what hbm_imm gives
 * on its context alone.  The contexts must be distinct and on one device; the
 * work runs on ctxs[0]'s stream, ordered after work already queued on each
 * context's own stream.  Outputs per instance i: seeds[i] int32[k_i] (host),
 * gains[i] uint64[k_i] (gains or gains[i] may be NULL), stats[i] (may be NULL),
 * status[i] (may be NULL).  Returns HBM_OK when every instance succeeded, else
 * the first failing instance's code (its outputs are untouched; its context's
 * last error tells why); device errors fail every instance. */
hbm_status hbm_imm_batch(hbm_ctx *const *ctxs, int32_t count, const hbm_query *queries, int32_t *const *seeds,
                         uint64_t *const *gains, hbm_imm_stats *stats, hbm_status *status);

/* ---------------------------------------------------------------- serving */

/* A request loop over one device-resident graph: queries are submitted at any
 * time and answered by a worker thread with continuous batching.  Each step of
 * the loop admits queued queries (arrival order) while fewer than max_active run
 * and the RR stores fit the budget, then advances every admitted query by one
 * IMM step in shared launches; a finished query frees its slot and store at once.
 * The sum of the admitted queries' store bytes is kept within store_budget:
 * sampling blocks are sized to the room left; when nothing can move the
 * youngest query is preempted (store dropped, re-queued at the head, recomputed
 * later with the same result).  A query that does not fit even alone fails with
 * HBM_EBUDGET.  Results are those of hbm_imm on the graph alone.
 * The server borrows the graph context's device graph and its encoding settings
 * (hbm_set_encoding) at creation: that context must not load another graph or be
 * destroyed while the server exists.  Server memory comes from hipMalloc; its
 * work runs on a stream of its own. */
typedef struct hbm_server hbm_server;

typedef struct hbm_serve_info {
    int32_t done;        /* 1 once the query finished (status holds the outcome) */
    hbm_status status;
    int32_t preemptions; /* times the query was preempted and restarted */
    double t_submit_ms;  /* server clock: ms since hbm_server_create */
    double t_admit_ms;   /* last admission (-1 while queued) */
    double t_done_ms;
    char error[128];
} hbm_serve_info;

typedef struct hbm_server_stats {
    int64_t submitted, admitted, completed, failed, preemptions;
    int64_t steps;            /* batched IMM steps run */
    int64_t peak_active;      /* most queries admitted at once */
    int64_t peak_store_bytes; /* most store bytes held at once (after a step) */
    int64_t active, queued;   /* now */
} hbm_server_stats;

/* HBM_EINVAL for a NULL argument, store_budget <= 0 or max_active < 1;
 * HBM_ESTATE if the context has no graph. */
hbm_status hbm_server_create(hbm_server **out, hbm_ctx *graph, int64_t store_budget, int32_t max_active);
/* Stops the loop after its current step; unfinished queries are dropped. */
void hbm_server_destroy(hbm_server *srv);
const char *hbm_server_last_error(const hbm_server *srv);
/* Queue a query; *ticket identifies it.  Invalid queries are accepted and fail at
 * admission (their status says why).  HBM_EDEVICE once the server has failed. */
hbm_status hbm_server_submit(hbm_server *srv, const hbm_query *q, int64_t *ticket);
/* State of a ticket (wait != 0 blocks until it finishes).  info->done = 0 while
 * pending.  Once done, seeds int32[k] / gains uint64[k] / stats (each may be NULL)
 * receive the result when info->status is HBM_OK, and the ticket is forgotten
 * (a later poll of it returns HBM_EINVAL).  HBM_EINVAL for an unknown ticket. */
hbm_status hbm_server_poll(hbm_server *srv, int64_t ticket, int32_t wait, int32_t *seeds, uint64_t *gains,
                           hbm_imm_stats *stats, hbm_serve_info *info);
/* Counters of the loop; HBM_EDEVICE (counters still filled) once it has failed. */
hbm_status hbm_server_get_stats(hbm_server *srv, hbm_server_stats *out);

/* ---------------------------------------------------------------- tuning */

/* Launch-shape parameters.  They change speed only, never results (RR sets are
 * pure functions of their index, selection is exact).  Unknown keys or values out
 * of range return HBM_EINVAL. */
typedef enum hbm_tune_key {
    HBM_TUNE_IC_TIER1 = 0,        /* 1: light IC sets on one wave each (default); 0: every set on a
                                     workgroup of its own */
    HBM_TUNE_IC_T1_BUDGET = 1,    /* edge groups (4 in-edges) one wave may expand before the set moves
                                     to a workgroup of its own; 0 = no limit.  Default 4096 */
    HBM_TUNE_BLOCK_SETS = 2,      /* RR sets sampled per block (scratch index size), >= 1024.
                                     Default 2^21 */
    HBM_TUNE_LT_PATH = 3,         /* LT walk length kept in LDS by one lane: 32 (default), 64, 128 or 256;
                                     longer walks move to device memory */
    HBM_TUNE_T2_QUEUE = 4,        /* queue entries of a big-set slot (>= 64, default 2^20); a set with
                                     more members is redone by a few slots with full-size queues */
    HBM_TUNE_T2_SLOTS = 5,        /* big-set workgroups per CU, 1..4 (default 4), each with its own
                                     visited bitmap and queue */
    HBM_TUNE_LDS_THREADS = 6,     /* threads of a workgroup of the LDS tier (IC sets past the wave
                                     budget, visited set and queue in LDS): 512, 1024, or 0 (default)
                                     = 1024 on graphs below 2^22 vertices, else 512 */
    HBM_TUNE_LDS_PER_CU = 7,      /* LDS-tier workgroups launched per CU, 1..4, or 0 (default) = 2
                                     on graphs below 2^22 vertices, else 3 */
    HBM_TUNE_SPARSE_COUNTS = 8,   /* greedy counts: 0 one per vertex; 1 one per vertex that occurs in
                                     the store (ids ascending, a vertex-to-slot map; the argmax reads
                                     the slots and one selection bit per vertex); 2 (default) = 1 on
                                     graphs of at least 2^22 vertices where the argmax then reads at
                                     most half as much, else 0.  Exact either way */
    HBM_TUNE_SELECT_GRAPH = 9,    /* 1: the greedy's k-iteration launch sequence (every instance of a
                                     batch) runs as a HIP graph: its launches read their arguments
                                     from a descriptor buffer and use grids that depend only on the
                                     store's shape (k, encoding, graph size), so a graph captured the
                                     first time a shape occurs is replayed for every later selection
                                     of that shape (up to 16 shapes kept per driving context).
                                     0 (default): launched kernel by kernel.  Not used while
                                     profiling */
    HBM_TUNE_SPILL_SLOTS = 10,    /* IC sets that outgrow an LDS tier: how many per sampling launch
                                     (0..4096, default 4096; set on the driving context, shared
                                     among a batch's instances in proportion to their lists) keep
                                     the BFS levels the tier completed (32 KB of device memory each,
                                     held by the driving context) so the next tier goes on from
                                     there; the rest start over from their root */
    HBM_TUNE_LDS_SMALL = 11,      /* IC: 1 puts an LDS tier of 1024 members (256 threads, four
                                     workgroups per CU) in front of the 2048-member one, which goes
                                     on from the levels it spilled (up to twice SPILL_SLOTS sets per
                                     block, 16 KB each); 0 does not; 2 (default) = 1 on graphs of at
                                     least 2^22 vertices, else 0 */
    HBM_TUNE_COUNT = 12
} hbm_tune_key;

hbm_status hbm_set_tuning(hbm_ctx *ctx, hbm_tune_key key, int64_t value);

/* Autotuner: picks the launch shapes for the given instances (one, or many as
 * hbm_imm_batch runs them) by timing whole IMM runs of the queries under candidate
 * settings, one key at a time (coordinate descent over BLOCK_SETS, IC_T1_BUDGET,
 * T2_SLOTS, LDS_THREADS, LDS_PER_CU and LT_PATH), and leaves the fastest applied to every context.  The
 * contexts' stores end up holding the probes' last run.  chosen int64[HBM_TUNE_COUNT]
 * (may be NULL) receives every key's setting, best_ms (may be NULL) the time of the
 * chosen one.  Results never depend on these settings.  Same argument rules as
 * hbm_imm_batch; a failing probe query returns its error. */
hbm_status hbm_autotune(hbm_ctx *const *ctxs, int32_t count, const hbm_query *queries, int64_t *chosen,
                        double *best_ms);

/* ---------------------------------------------------------------- profiling */

/* Per-kernel statistics gathered while profiling is on: every launch is timed
 * with a pair of HIP events recorded on the context's stream.  alg_bytes and
 * alg_ops are the algorithmic traffic and work of those launches (the bytes the
 * method must move, excluding re-reads; ops = Philox calls for samplers), from
 * device-side counters where the amount depends on the data. */
typedef struct hbm_kernel_stat {
    char name[32];
    int64_t launches;
    double total_ms;
    double alg_bytes;
    double alg_ops;
} hbm_kernel_stat;

/* enable != 0 starts profiling and clears the statistics; 0 stops it. */
hbm_status hbm_profile(hbm_ctx *ctx, int32_t enable);

/* Copy up to `cap` entries into host `out`; *count gets the number available. */
hbm_status hbm_profile_read(hbm_ctx *ctx, hbm_kernel_stat *out, int32_t cap, int32_t *count);

/* Device memory held by the context (graph, store, sampling and selection scratch,
 * descriptors; the fixed array of hbm_select_seeds_noalloc is not counted): *bytes_now
 * now, *bytes_peak the most at any moment since creation or the last reset.  The
 * paper's memory tables report peak memory; this is the device-side figure.
 * reset_peak != 0 sets the peak to the current bytes after reading it. */
hbm_status hbm_get_memory(hbm_ctx *ctx, int64_t *bytes_now, int64_t *bytes_peak, int32_t reset_peak);

/* Throughput probe of the RNG the samplers use (Philox4x32-10, the same device
 * function): `blocks` workgroups of 256 threads each draw calls_per_thread outputs
 * (even, >= 2) from counters of their own.  *ms gets the kernel time (HIP events on
 * the context's stream), *checksum a sum of the outputs (the same for the same
 * arguments).  Calls per second = blocks * 256 * calls_per_thread / ms * 1e3. */
hbm_status hbm_bench_philox(hbm_ctx *ctx, int64_t calls_per_thread, int32_t blocks, double *ms, uint32_t *checksum);

/* ---------------------------------------------------------------- inspection */

/* Decode RR set j to ascending ids in host `buf` (capacity `cap`); *len gets
 * its size.  HBM_EINVAL if j is out of range or cap is too small (then *len
 * still gets the size). */
hbm_status hbm_get_rr(hbm_ctx *ctx, int64_t j, int32_t *buf, int64_t cap, int64_t *len);

/* Decode sets [j0, j1) into host arrays: off int64[j1-j0+1] (relative offsets)
 * and mem int32[cap].  *total gets the member count; HBM_EINVAL if cap is too small. */
hbm_status hbm_dump_sets(hbm_ctx *ctx, int64_t j0, int64_t j1, int64_t *off, int32_t *mem, int64_t cap,
                         int64_t *total);

/* Sizes and coding statistics of the store. */
hbm_status hbm_get_store_stats(hbm_ctx *ctx, hbm_store_stats *out);

/* Raw arrays of the store and the graph, copied to host, for bit-level checks.
 * `what` selects the array; *bytes gets its size; HBM_EINVAL if cap is too
 * small or the array does not exist for the current encoding. */
typedef enum hbm_array {
    HBM_A_IN_PTR = 0,    /* int64[n+1]  transposed-graph offsets */
    HBM_A_IN_SRC = 1,    /* int32[m]    in-edge sources */
    HBM_A_THRESH = 2,    /* uint32[m or n]  live thresholds: edge live iff (philox word >> 8) < thr */
    HBM_A_COUNTS = 3,    /* uint32[n]   vertex frequencies over the whole store */
    HBM_A_WARM = 4,      /* uint32[n]   vertex frequencies over the warm-up block */
    HBM_A_HOT = 5,       /* int32[nhot] hot vertices by rank */
    HBM_A_BITMAP = 6,    /* uint64[ceil(nsets/64) * nhot], word-major: word w, rank r at w*nhot + r */
    HBM_A_RAW_OFF = 7,   /* int64[nsets+1] offsets of the plain ids */
    HBM_A_RAW_MEM = 8,   /* int32[]     plain ids, ascending per set */
    HBM_A_LENS = 9,      /* uint8[n]    Huffman code lengths (0 = codeless) */
    HBM_A_CODES = 10,    /* uint32[n]   canonical codes, right-aligned */
    HBM_A_BITOFF = 11,   /* int64[nsets+1] start bit of each set's string */
    HBM_A_PAYLOAD = 12,  /* uint32[]    bit stream, MSB first within each word */
    HBM_A_ARR_HOT = 13,  /* int32[nar]  vertices with array rows, in hot order */
    HBM_A_ARR_OFF = 14,  /* int64[ceil(nsets/2^16) * (nar+1)] chunk-major offsets into ARR_LOW */
    HBM_A_ARR_LOW = 15   /* uint16[]    ascending set offsets (j mod 2^16) per (chunk, row) */
} hbm_array;

hbm_status hbm_export(hbm_ctx *ctx, hbm_array what, void *host_out, int64_t cap_bytes, int64_t *bytes);

/* Library version string. */
const char *hbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HBMAX_H */
