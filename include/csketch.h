/*
 * csketch.h - C ABI of the MI355X (gfx950) convolution Count sketch library.
 *
 * Method: Heddes, Nunes, Givargis & Nicolau, "Convolution and Cross-Correlation of
 * Count Sketches Enables Fast Cardinality Estimation of Multi-Join Queries"
 * (SIGMOD 2024).  One Count sketch per relation of a join query, d independent
 * repetitions of m int64 counters each.  A tuple adds its frequency change, times the
 * product of the sign hashes of the joins its attributes take part in, to the counter
 * at the sum (mod m) of its attributes' bin hashes (Sec. 3.2, Eq. 2-4, Alg. 2).  The
 * estimate of the join size combines the sketches along the join graph by circular
 * cross-correlation and Hadamard products (Eq. 5, Alg. 3) and takes the median of the
 * d repetitions (Sec. 3.3).
 *
 * Conventions (the paper leaves them open; this library fixes them):
 *   - hash field p = 2^61 - 1; keys are uint32, so distinct keys stay distinct mod p;
 *   - coefficients come from SplitMix64 seeded with `seed`: each draw is next() >> 3,
 *     redrawn if it equals p; draw order: for each repetition t, for each join e (in
 *     the caller's edge order) a0, a1, a2, a3; then for each graph component q
 *     (numbered by smallest attribute id) b0, b1;
 *   - sign s_e(x) = +1 if (a0 + a1 x + a2 x^2 + a3 x^3 mod p) is even, else -1
 *     (4-wise independent family); bin h_q(x) = (b0 + b1 x mod p) mod m (2-wise);
 *   - counters are int64 and wrap modulo 2^64;
 *   - the median of an even number of repetitions is the lower middle value.
 *
 * Memory: every pointer documented as "device" must be device memory of the device
 * that was current when the handle was created (e.g. a torch CUDA/HIP tensor's
 * data_ptr()).  Streams are hipStream_t values passed as void* (NULL = null stream).
 * The library allocates and owns the counters and its work buffers; callers own
 * every buffer they pass in and keep it alive until the stream has passed the call.
 *
 * Errors: every call returns a cs_status; on failure cs_last_error() returns a
 * thread-local message.  No exception crosses this boundary.  Handles are not
 * thread-safe: one thread at a time per handle.
 */
#ifndef CSKETCH_H
#define CSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cs_status {
    CS_OK = 0,
    CS_EINVAL = 1,   /* bad argument (null pointer, size out of range, bad relation id) */
    CS_EGRAPH = 2,   /* the join graph is not an acyclic connected equi-join query */
    CS_ENOMEM = 3,   /* device or host allocation failed */
    CS_EDEVICE = 4,  /* a HIP runtime call failed */
    CS_EBUSY = 5,    /* admission refused: memory budget or queue full */
    CS_ERANGE = 6    /* a value is beyond what the library represents */
} cs_status;

/* A join query (Sec. 2.6, Fig. 3).  Attributes 0..n_attr-1 are globally numbered
 * vertices; attr_rel[u] is the relation owning attribute u; edges[2e], edges[2e+1]
 * are the attributes joined by join e.  Valid queries: every relation owns at least
 * one attribute, every attribute takes part in at least one join, a join links two
 * different relations, and the relations with the joins form a tree (n_edge =
 * n_rel - 1, connected).  Self-joins are written with a copy of the relation.
 * Limits: n_rel <= 16, n_attr <= 32, at most 8 attributes per relation, at most 8
 * joins per attribute.  All arrays are host memory, read during the call only. */
typedef struct cs_graph {
    int32_t n_rel;
    int32_t n_attr;
    const int32_t *attr_rel;   /* [n_attr] */
    int32_t n_edge;
    const int32_t *edges;      /* [n_edge][2] */
} cs_graph;

typedef struct cs_sketch cs_sketch;   /* opaque: the sketches of one query */

/* Result of an estimate.  `value` is the median over the d repetitions as fp64: the
 * correctly rounded value of the exact integer median when exact != 0.  value_i64
 * holds the exact median when exact != 0 and it fits in int64 (fits_i64 != 0). */
typedef struct cs_estimate_t {
    double value;
    int64_t value_i64;
    int32_t exact;
    int32_t fits_i64;
    int32_t d;
    int32_t n_modular;   /* repetitions whose exact value needed the modular path */
} cs_estimate_t;

/* Per-repetition detail, for tests and diagnostics (host arrays of length d). */
typedef struct cs_reps_t {
    double *value;       /* X_t as fp64 (correctly rounded when exact) */
    int64_t *lo;         /* low 64 bits of the exact X_t (two's complement int128) */
    int64_t *hi;         /* high 64 bits of the exact X_t */
    int32_t *exact;      /* 1: lo/hi hold X_t exactly */
    double *bound;       /* certified bound on |fp64 FFT estimate - X_t| (0 if no FFT) */
} cs_reps_t;

/* Update strategies (all give bit-identical counters). */
typedef enum cs_update_strategy {
    CS_UPDATE_AUTO = 0,           /* the autotuner's choice when it has one for this class;
                                     else global atomics below 65536 tuple-repetitions,
                                     PARTITION beyond 2^16 buckets (weights NULL or +-1,
                                     <= 2 columns) except LDS_PRIVATE at m = 2^17 with
                                     d <= 9 and every column in one join,
                                     WAVE_AGGREGATE beyond 2^18 buckets with general
                                     weights, LDS_PRIVATE otherwise */
    CS_UPDATE_GLOBAL_ATOMIC = 1,  /* one device-scope int64 atomic per tuple and repetition */
    CS_UPDATE_LDS_PRIVATE = 2,    /* the d x m counters cut into LDS-sized segments;
                                     each workgroup accumulates one segment for one chunk
                                     of tuples in LDS, stores partial sums to the
                                     handle's scratch buffer, and a reduce kernel adds
                                     them into the counters */
    CS_UPDATE_WAVE_AGGREGATE = 3, /* equal buckets of one wavefront merged before the atomic */
    CS_UPDATE_PARTITION = 4       /* sort by bucket range: every tuple hashed once per
                                     repetition into a 16-bit record, grouped by
                                     (repetition, range of 2^14 buckets) per block of
                                     4096 tuples (up to eight hot tuples per block,
                                     candidates seeded by the relation's hottest tuples
                                     of its previous call, summed instead), then one
                                     workgroup per group sums its records in LDS and owns
                                     those counters; needs weights NULL or
                                     CS_UPDATE_UNIT_WEIGHTS, <= 2 columns */
} cs_update_strategy;

/* cs_update_ex flags */
#define CS_UPDATE_UNIT_WEIGHTS 1  /* the caller guarantees every weight is +1 or -1 */
#define CS_UPDATE_NO_COMPACT 2    /* segmented strategy: do not use the compacting kernel for
                                     bucket-range segments (testing and tuning) */
#define CS_UPDATE_NO_COUNTERS16 4 /* segmented strategy: do not use 16-bit LDS counters
                                     (testing and tuning) */
#define CS_UPDATE_TEST_FULL_REDUCTION 8 /* testing: most tuples take the full mod-p
                                     reduction of their hashes, which otherwise only
                                     hashes within 3 of a multiple of 2^61 - 1 need
                                     (the counters are the same) */

/* Estimate plans chosen at cs_create from the join graph. */
typedef enum cs_plan_kind {
    CS_PLAN_DOT = 1,       /* two relations: X_t = <c_0, c_1> in exact 128-bit integers */
    CS_PLAN_SPECTRAL = 2,  /* every graph component joins exactly two attributes (chains,
                              stars, any tree of binary joins): X_t = (1/m) sum_f of the
                              product of the relations' spectra, conjugated on alternate
                              levels; fp64 FFT + modular residue for exactness */
    CS_PLAN_GENERAL = 3    /* some component joins three or more attributes: Alg. 3's
                              Hadamard / cross-correlation sequence in modular arithmetic
                              (number-theoretic transforms), exact */
} cs_plan_kind;

typedef struct cs_info_t {
    int32_t n_rel, n_attr, n_edge, n_comp;
    uint32_t m, d;
    int32_t plan;              /* cs_plan_kind */
    int32_t device;
    uint64_t counter_bytes;    /* r * d * m * 8 */
    uint64_t workspace_bytes;  /* estimate work buffers currently held */
} cs_info_t;

/* ------------------------------------------------------------------ lifecycle */

/* Validate the query, draw the hash coefficients (Alg. 1: SampleSignHashes and
 * SampleBinHashes; Sec. 3.2 initialization), allocate r*d*m int64 counters on the
 * current device and zero them.  2 <= m <= 2^20 (any m: buckets are h(x) mod m; a
 * power of two unlocks the spectral plan, the partition strategy and the one-join
 * kernels, an even m the 16-bit counters); 1 <= d <= 64.  With m not a power of two a
 * graph of binary joins (r > 2) is estimated by the general plan.
 * Errors: CS_EINVAL, CS_EGRAPH, CS_ENOMEM, CS_EDEVICE. */
cs_status cs_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed,
                    cs_sketch **out);

/* Free the handle and its device memory (synchronises the device first). */
cs_status cs_destroy(cs_sketch *h);

/* Bytes of counters cs_create would allocate (for admission control); 0 if invalid. */
uint64_t cs_sketch_bytes(const cs_graph *graph, uint32_t m, uint32_t d);

cs_status cs_get_info(const cs_sketch *h, cs_info_t *out);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *cs_last_error(void);

/* ------------------------------------------------------------------ update (Alg. 2) */

/* Stream n tuples of relation `rel` into its sketch (Alg. 2 for each repetition;
 * Eq. 2-4 define the counters it produces).
 * Calls on one handle must be ordered (one stream, or event dependencies).  The
 * segmented and partition strategies use the handle's own scratch buffer (partial sums,
 * records), never another handle's: the first update that needs it allocates it, sized
 * for that call (at most ~67 MB, depending on m, d, n and the weight kind), after
 * waiting for `stream`; a later call that can use more grows it the same way; every
 * other call allocates nothing and never waits on the host (cs_update_noalloc never
 * allocates).
 *   keys:    device (or pinned / managed host) memory, uint32 [n][a_rel] tuple-major;
 *            column c is the c-th attribute of `rel` in ascending attribute id.
 *   weights: the same kinds of memory, int64 [n] frequency changes Delta (turnstile
 *            model, Sec. 2.1), or NULL for Delta = +1.
 * Asynchronous and ordered on `stream`.  n = 0 is a no-op.
 * Errors: CS_EINVAL (bad handle, rel out of range, keys NULL with n > 0, keys or weights
 * in memory the device cannot read, such as pageable host memory: checked on the host
 * before anything is enqueued), CS_ENOMEM (the scratch buffer). */
cs_status cs_update(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                    uint64_t n, void *stream);

/* Same with an explicit strategy and launch width (0 = automatic); for tests and
 * tuning.  grid_blocks is the number of workgroups for the atomic strategies and the
 * number of tuple chunks for the segmented one (bounded by its scratch buffer).
 * CS_EINVAL if the strategy does not support this handle's m and d. */
cs_status cs_update_ex(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                       uint64_t n, void *stream, int32_t strategy, int32_t grid_blocks,
                       int32_t flags);

/* cs_update_ex that also records two caller-created hipEvent_t on `stream`: ev_start just
 * before the update's hashing kernel and ev_stop just after it (the segmented strategy's
 * reduction of partial sums and the partition strategy's accumulation pass fall outside;
 * a partition update of more than 2^23 tuples runs in chunks, and then both passes of
 * every chunk fall inside).  Either event may be NULL.  Per-kernel timing for monitoring
 * and tuning; the counters are the same as cs_update's.  Errors as cs_update_ex, and
 * CS_EDEVICE if an event cannot be recorded. */
cs_status cs_update_timed(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                          uint64_t n, void *stream, int32_t strategy, int32_t grid_blocks,
                          int32_t flags, void *ev_start, void *ev_stop);

/* cs_update for callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * counters as cs_update (automatic strategy), but the strategies' scratch buffer
 * (partial sums, records) is a file-scope device array of
 * cs_update_noalloc_scratch_bytes() bytes (64 MiB) that each GPU holds until the process
 * ends, instead of the handle's.  The call allocates nothing (no hipMalloc / hipFree, no
 * allocating library routine).
 *   flags: 0 or CS_UPDATE_UNIT_WEIGHTS.  Other arguments as cs_update.
 * The handle's device must be the current device.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams without an ordering
 * between them, or several host threads) race on it and must be ordered by the caller;
 * consecutive calls on one stream are ordered by it.  Nothing the array keeps from an
 * earlier call is read.
 * Errors: as cs_update, and CS_EINVAL when the strategy for this (m, d) would need more
 * scratch than the array holds (e.g. general weights with d * m beyond 2^23 counters),
 * refused before anything is enqueued. */
cs_status cs_update_noalloc(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                            uint64_t n, int32_t flags, void *stream);
size_t cs_update_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------ machine-balance probes */

/* The two rates the update is compared with, measured on the current device (the
 * update's hashes are Horner steps v <- v * x + a mod 2^61 - 1, Sec. 4; Alg. 2):
 * cs_k0_horner runs a kernel of nothing but independent Horner steps (the library's own
 * step, 16 wavefronts per CU, 8 chains per lane, `iters` steps per chain) and returns
 * steps per second; cs_k0_stream_read reads `bytes` of device memory at `buf` (caller
 * owned, at least 16 bytes) `passes` times and returns bytes per second.  Synchronous
 * (null stream); each allocates and frees a small output buffer.  Benchmarking only.
 * Errors: CS_EINVAL (bad arguments, memory the device cannot read), CS_EDEVICE. */
cs_status cs_k0_horner(uint64_t iters, double *steps_per_s);
cs_status cs_k0_stream_read(const void *buf, uint64_t bytes, int32_t passes, double *bytes_per_s);

/* ------------------------------------------------------------------ filtered ingestion */

#define CS_MAX_PREDICATES 8

/* One range predicate on a non-join attribute column: lo <= value <= hi (uint32).  An
 * equality is lo == hi; a one-sided bound uses 0 or 0xFFFFFFFF. */
typedef struct cs_predicate {
    int32_t column;            /* column of the attrs buffer */
    uint32_t lo, hi;
} cs_predicate;

/* cs_update restricted to the tuples that satisfy every predicate (a conjunction): the
 * query's filters applied while its relation streams in, so tuples that fail them never
 * reach the sketch (the experimental setup of Sec. 4.1).
 *   attrs: device, uint32 [n][n_attrs] tuple-major, the tuples' filtered columns
 *          (1 <= n_attrs <= CS_MAX_PREDICATES); may be NULL when n_preds = 0.
 *   preds: host array of n_preds (0..CS_MAX_PREDICATES) predicates.
 *   flags: as cs_update_ex (CS_UPDATE_UNIT_WEIGHTS ...).
 *   n_kept: optional.  NULL: the call is asynchronous and ordered on `stream` like
 *           cs_update.  Non-NULL: the kernels also count the tuples that passed and the
 *           call waits on `stream` for that count.
 * Nothing is read back unless n_kept asks for the count.  When every key column takes
 * part in one join, m is a power of two, the Deltas are +-1 and the relation has at
 * most two key columns: for m in (2^15, 2^16] one compaction pass evaluates the
 * predicates once per tuple and writes the kept tuples' keys into a buffer of the
 * handle (in rounds of 2^23 or 2^24 tuples), and the 16-bit update reads their count on
 * the device -- that buffer (partial sums plus a round, about 160 MB at d = 9) is
 * allocated by the handle's first filtered update for m in (2^15, 2^16], after waiting
 * for `stream`, and kept until cs_destroy; nothing else is allocated.  Beyond 2^16
 * buckets the partition strategy's hashing pass evaluates the predicates itself and
 * compacts the kept tuples in LDS before hashing.  Every other shape takes global
 * atomics that skip the tuples failing the predicates.
 * Errors: CS_EINVAL (arguments), CS_ENOMEM, CS_EDEVICE. */
cs_status cs_update_filtered(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                             uint64_t n, const uint32_t *attrs, int32_t n_attrs,
                             const cs_predicate *preds, int32_t n_preds, int32_t flags, void *stream,
                             uint64_t *n_kept);

/* ------------------------------------------------------------------ autotuner */

#define CS_TUNE_MAX_CANDIDATES 16
/* Strategy codes of tuning-table entries that are not cs_update strategies (they appear
 * in files written by cs_tune_save): a batched task class's kind, and a transform
 * length's split. */
#define CS_TUNE_BATCH_ATOMIC 16
#define CS_TUNE_BATCH_SEGMENT 17
#define CS_TUNE_BATCH_SORT 18
#define CS_TUNE_TRANSFORM_SPLIT 32

typedef struct cs_tune_candidate {
    int32_t strategy;          /* cs_update_strategy */
    int32_t grid_blocks;       /* as in cs_update_ex (0 = automatic) */
    int32_t flags;             /* CS_UPDATE_NO_COMPACT / CS_UPDATE_NO_COUNTERS16 */
    int32_t valid;             /* 1: ran, counters equal the reference's; 0: not
                                  applicable to this handle; -1: counters differed */
    float ms;                  /* median of three timed runs, -1 if not valid */
} cs_tune_candidate;

typedef struct cs_tune_report {
    int32_t n;                 /* candidates tried */
    int32_t best;              /* index of the chosen one */
    cs_tune_candidate cand[CS_TUNE_MAX_CANDIDATES];
} cs_tune_report;

/* Times every applicable update variant (strategy, launch width, kernel flags) on these
 * tuples of relation `rel` (same arguments as cs_update; `flags` may carry
 * CS_UPDATE_UNIT_WEIGHTS), each into private counters so the handle's sketch is left
 * untouched, checks each variant's counters against the global-atomic kernel's
 * (a variant that differs is never chosen), and records the fastest for this class:
 * (device architecture, m, d, key columns, one-join columns or not, weight kind,
 * floor(log2 n)).  cs_update / cs_update_ex with CS_UPDATE_AUTO then use it for every
 * handle of that class.  Synchronous; allocates two d x m int64 buffers for its run.
 * Errors: CS_EINVAL (arguments), CS_ENOMEM, CS_EDEVICE. */
cs_status cs_tune_update(cs_sketch *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                         uint64_t n, void *stream, int32_t flags, cs_tune_report *out);
/* Forget every tuned choice. */
cs_status cs_tune_clear(void);
/* Write the tuned choices to a text file / merge those of a file written by
 * cs_tune_save (CS_EINVAL if unreadable or malformed; nothing is merged then). */
cs_status cs_tune_save(const char *path);
cs_status cs_tune_load(const char *path);
/* Number of tuned classes held. */
cs_status cs_tune_count(int32_t *n_out);

/* ------------------------------------------------------------------ estimate (Eq. 5, Alg. 3) */

/* Estimate the join size: per repetition X_t (Eq. 5, evaluated as in Alg. 3), then
 * the median.  Runs on `stream` and blocks until the result is on the host.
 * `reps` may be NULL.  Errors: CS_EINVAL, CS_EDEVICE, CS_ENOMEM. */
cs_status cs_estimate(cs_sketch *h, void *stream, cs_estimate_t *out, const cs_reps_t *reps);

/* Asynchronous estimate: the same result as cs_estimate (Eq. 5 per repetition through
 * Alg. 3, median over the repetitions, Sec. 3.3), with the whole computation enqueued on
 * `stream` and the result written to *out, which must be memory the device can write
 * (device memory, or pinned host memory from hipHostMalloc), once the stream passes the
 * call; the call returns without waiting.  No host round trip happens, so a repetition
 * that needs more primes than the speculative modular step computes (as many as the
 * handle's last synchronous estimate needed, at most 5 = about 155 bits of window; 5
 * before the first) keeps its fp64 value, and out->exact is then 0.  Stream-ordered
 * with the handle's updates and estimates; calls on other streams must not overlap it.
 * Errors (returned at once, nothing enqueued): CS_EINVAL for queries with the general
 * plan (their estimate needs host round trips) and for an `out` that is not device
 * memory of the handle's device or pinned / managed host memory. */
cs_status cs_estimate_async(cs_sketch *h, void *stream, cs_estimate_t *out);

/* ------------------------------------------------------------------ batched mode */

/* One relation's tuple stream within a batch (same meaning as cs_update's arguments). */
typedef struct cs_update_item {
    cs_sketch *sketch;
    int32_t rel;
    int32_t flags;             /* CS_UPDATE_UNIT_WEIGHTS or 0 */
    const uint32_t *keys;      /* device, [n][a_rel] */
    const int64_t *weights;    /* device, [n], or NULL for +1 */
    uint64_t n;
} cs_update_item;

typedef struct cs_batch cs_batch;   /* work-list tables, estimate workspace, captured graph */

cs_status cs_batch_create(cs_batch **out);
cs_status cs_batch_destroy(cs_batch *b);

/* Alg. 2 for many queries' relations in ONE persistent kernel launch: the items are
 * cut into tasks (tuple ranges; for relations with many tuples per counter, one LDS
 * segment of the counters each), ordered largest first and pulled by one 1024-thread
 * workgroup per CU.  Counters end bit-identical to cs_update of every item.  Items
 * may belong to different handles (different graphs, m, d) on one device; two items
 * must not target one relation of one handle twice unless ordered by the caller's
 * stream.  Plans the work list on the host, uploads it, launches, returns without
 * waiting.  Errors: CS_EINVAL (bad item), CS_ENOMEM, CS_EDEVICE. */
cs_status cs_batch_update(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream);

/* Plan the items once and capture the launch (counter reset + persistent kernel) in a
 * HIP graph; cs_batch_replay launches it again on `stream` with the same buffers. */
cs_status cs_batch_capture(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream);
cs_status cs_batch_replay(cs_batch *b, void *stream);

/* Estimates of n queries at once (Eq. 5 / Alg. 3 + median per query): one norm launch,
 * one FFT and one product-reduce launch per sketch length, one finalize launch, plus
 * the modular exactness pass for the repetitions that need it.  Results are identical
 * to cs_estimate of each query.  outs[n]; reps NULL or n entries.  Blocking. */
cs_status cs_batch_estimate(cs_batch *b, cs_sketch *const *sketches, int32_t n, void *stream,
                            cs_estimate_t *outs, const cs_reps_t *reps);

/* Task counts of the last planned batch update. */
cs_status cs_batch_stats(const cs_batch *b, uint64_t *tasks_atomic, uint64_t *tasks_segment);
/* The same with the sort-reduce tasks counted apart (each pointer may be NULL). */
cs_status cs_batch_task_counts(const cs_batch *b, uint64_t *tasks_atomic, uint64_t *tasks_segment,
                               uint64_t *tasks_sort_reduce);

/* Autotuner of the batched update's tasks: the items are grouped into classes (m, d,
 * key columns, one-join columns, unit weights, floor(log2 n)), and for each class the
 * class's items alone run as one persistent launch with every task choice -- global
 * atomics; sort-reduce (per repetition, each wavefront sorts the counter indices of its
 * 64 tuples, sums the runs of equal ones and adds each run with one global atomic); or
 * LDS segments over tuple chunks of 2^14, 2^16, 2^18 or 2^20 -- into private
 * counters (the handles' sketches are left untouched); a choice whose counters differ
 * from the global-atomic run's is never taken.  Each choice is then timed (median of
 * three) on enough copies of the class's work, each into its own counters, to fill the
 * chip, so that the time per copy is the class's cost inside a large batch; the fastest
 * is stored in the tuning table, and cs_batch_update / cs_batch_capture plan that class
 * with it from then on (cs_tune_save / cs_tune_load persist it).  The fixed rule the
 * planner otherwise uses is timed beside them.  Synchronous; allocates two buffers of
 * the largest class's counters and up to 1 GiB for the copies.
 * Errors: CS_EINVAL, CS_ENOMEM, CS_EDEVICE. */
typedef struct cs_tune_batch_report {
    int32_t classes;   /* classes tuned */
    int32_t rejected;  /* candidate runs whose counters differed from the reference */
    float rule_ms;     /* sum over classes of the fixed rule's time per copy */
    float tuned_ms;    /* sum over classes of the chosen candidate's time per copy */
} cs_tune_batch_report;
cs_status cs_tune_batch_update(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream,
                               cs_tune_batch_report *out);

/* Autotuner of the two-pass transforms (lengths 2^13..2^21) the estimate runs: for each
 * row length 2^S (S = 10..12 with S < log2m <= 2S) it times the fp64 FFT and one
 * prime's number-theoretic transform of n_vec synthetic vectors of length 2^log2m,
 * checks that the number-theoretic spectrum equals the default split's at every
 * frequency (exact arithmetic; the split only permutes the output), and stores the
 * fastest for this device and length: later estimates of that length use it (an
 * estimate in flight keeps the split it started with).  out->cand[i].grid_blocks holds
 * S, .ms the median of three runs.  Synchronous.  Errors: CS_EINVAL (log2m outside
 * 13..21, n_vec outside 1..4096), CS_ENOMEM, CS_EDEVICE. */
cs_status cs_tune_transform(int32_t log2m, int32_t n_vec, void *stream, cs_tune_report *out);

/* ------------------------------------------------------------------ serving */

typedef struct cs_server_config {
    uint64_t memory_budget;    /* bytes of counters admitted over all live queries (0: none) */
    int32_t n_streams;         /* update streams (default 2) */
    int32_t max_batch_items;   /* update items per launch (default 4096) */
    int32_t max_pending;       /* submitted-but-unfinished requests before CS_EBUSY (0: none) */
    int32_t reserved;
} cs_server_config;

typedef struct cs_completion {
    uint64_t ticket;
    int32_t qid;
    int32_t kind;              /* 0 update, 1 estimate */
    int32_t status;            /* cs_status of the request */
    int32_t reserved;
    double submit_us, start_us, done_us;   /* host steady-clock microseconds */
    cs_estimate_t estimate;    /* kind 1 */
} cs_completion;

typedef struct cs_server_stats_t {
    uint64_t submitted, completed, used_bytes;
    uint64_t update_launches, estimate_batches, epochs;
    int32_t live_queries;
    int32_t reserved;
} cs_server_stats_t;

typedef struct cs_server cs_server;

/* A server keeps live sketches resident on the current device and executes update
 * batches and estimate requests as they arrive: updates of each arrival epoch go into
 * one batched persistent launch (round robin over n_streams), estimates into one
 * batched estimate on their own stream, overlapping with later updates.  An estimate
 * of a query reflects exactly the updates of that query submitted before it.  Two
 * native threads (scheduler, estimator). */
cs_status cs_server_create(const cs_server_config *cfg, cs_server **out);
/* Waits for all submitted requests, stops the threads, frees every live query. */
cs_status cs_server_destroy(cs_server *s);
/* Admission: CS_EBUSY when the query's counters do not fit the memory budget. */
cs_status cs_server_add_query(cs_server *s, const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed,
                              int32_t *qid);
/* Marks the query removed at once (later submissions for it are refused with
 * CS_EINVAL; its requests still queued complete with CS_EINVAL), waits for this query's
 * own requests already on the GPU, then frees its memory.  Requests of other queries keep
 * flowing meanwhile.  A second removal of the same qid returns CS_EINVAL. */
cs_status cs_server_remove_query(cs_server *s, int32_t qid);
/* The handle of a live query (for reading its sketches; do not update it directly). */
cs_status cs_server_sketch(cs_server *s, int32_t qid, cs_sketch **out);
/* Enqueue a turnstile update batch (device keys / weights owned by the caller, alive
 * until its completion is polled) or an estimate request; returns a ticket.
 * CS_EBUSY when max_pending requests are outstanding. */
cs_status cs_server_submit_update(cs_server *s, int32_t qid, int32_t rel, const uint32_t *keys,
                                  const int64_t *weights, uint64_t n, int32_t flags, uint64_t *ticket);
cs_status cs_server_submit_estimate(cs_server *s, int32_t qid, uint64_t *ticket);
/* Non-blocking: move up to max finished requests into out. */
cs_status cs_server_poll(cs_server *s, cs_completion *out, int32_t max, int32_t *n_out);
/* Block until every submitted request has finished. */
cs_status cs_server_drain(cs_server *s);
cs_status cs_server_stats(cs_server *s, cs_server_stats_t *out);

/* ------------------------------------------------------------------ state */

/* Zero every counter (stream-ordered). */
cs_status cs_reset(cs_sketch *h, void *stream);

/* dst += src counter-wise (sketch linearity, Sec. 2.2).  Both handles must have the
 * same graph, m, d and seed.  Stream-ordered. */
cs_status cs_merge(cs_sketch *dst, const cs_sketch *src, void *stream);

/* Copy relation rel's counters, int64 [d][m], to host memory (synchronous). */
cs_status cs_read_sketch(cs_sketch *h, int32_t rel, int64_t *host_out);

/* Device address of relation rel's counters, int64 [d][m] (owned by the handle). */
cs_status cs_sketch_device_ptr(cs_sketch *h, int32_t rel, int64_t **out);

/* Copy the drawn coefficients to host memory: sign [d][n_edge][4] (a0..a3), bin
 * [d][n_comp][2] (b0, b1). */
cs_status cs_read_coeffs(const cs_sketch *h, uint64_t *sign_out, uint64_t *bin_out);

/* Graph component of each attribute, int32 [n_attr] (host). */
cs_status cs_read_components(const cs_sketch *h, int32_t *psi_out);

/* ------------------------------------------------------------------ checkpoint and resume */

/* A sketch is its counters plus what draws its hash functions (graph, m, d, seed), so a
 * checkpoint re-creates an identical handle, and by linearity (Sec. 2.2) updates after a
 * resume give the counters an uninterrupted run would have.
 *   cs_export: *needed = blob size; when buf is not NULL and cap >= *needed, writes the
 *              blob to host memory buf (synchronises the device).  Blob: "CSKETCH1",
 *              uint32 version 1, m, d, n_rel, n_attr, n_edge, uint64 seed, int32
 *              attr_rel[n_attr], int32 edges[n_edge][2], int64 counters[n_rel][d][m],
 *              uint64 FNV-1a of every preceding byte; little-endian.
 *   cs_import: validates the blob (magic, version, ranges, length, checksum: CS_EINVAL
 *              before any device work when it fails), creates the handle on the current
 *              device and uploads the counters. */
cs_status cs_export(cs_sketch *h, void *buf, size_t cap, size_t *needed);
cs_status cs_import(const void *buf, size_t len, cs_sketch **out);

/* ------------------------------------------------------------------ timing */

/* Timing events (hipEvent_t) for cs_update_timed and for marks between calls, created
 * without the system-scope fence an ordinary event performs when it completes, so that
 * recording one does not write back and invalidate caches in the middle of the timed
 * work.  Not for synchronising with host reads of device memory.
 *   cs_timer_create:  *ev receives a new event (CS_EDEVICE on failure).
 *   cs_timer_record:  records ev on `stream` (stream-ordered).
 *   cs_timer_elapsed: waits for `stop`, then *ms = time from start to stop.
 *   cs_timer_destroy: releases ev. */
cs_status cs_timer_create(void **ev);
cs_status cs_timer_record(void *ev, void *stream);
cs_status cs_timer_elapsed(void *start, void *stop, float *ms);
cs_status cs_timer_destroy(void *ev);

/* ------------------------------------------------------------------ per-attribute sketches */

/* Sketches kept per attribute for query optimizers (Sec. 3.4): the sizes of many
 * sub-queries are needed, and an attribute's sketch can serve every sub-query that joins
 * the attribute once.  Every attribute u of `graph` gets one Count sketch int64 [d][m]
 * built with the hash functions of its graph component Psi(u) (per repetition a degree-3
 * sign polynomial and a degree-1 bin polynomial, drawn from the seeded SplitMix64 stream
 * in the order t, component, a0..a3, b0, b1), so the two-relation join of any two
 * attributes of one component is estimated from their two sketches.  For a graph with one
 * join the sketches are those cs_create draws for it. */
typedef struct cs_attr cs_attr;  /* opaque */

/* As cs_create (2 <= m <= 2^20 any m, 1 <= d <= 64); allocates w*d*m int64 counters.
 * Errors: CS_EINVAL, CS_EGRAPH, CS_ENOMEM, CS_EDEVICE. */
cs_status cs_attr_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, cs_attr **out);

/* Free the handle (synchronises the device first). */
cs_status cs_attr_destroy(cs_attr *h);

/* One pass over n tuples of relation rel (keys uint32 [n][a_rel], tuple-major, device;
 * weights int64 [n] or NULL for Delta = +1; flags: CS_UPDATE_UNIT_WEIGHTS): the sketch of
 * every attribute of rel is updated (Alg. 2 with one column and one join).  Stream-
 * ordered; calls on one handle from different streams must not overlap (they share a
 * column buffer). */
cs_status cs_attr_update(cs_attr *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                         uint64_t n, int32_t flags, void *stream);

/* Zero every counter (stream-ordered). */
cs_status cs_attr_reset(cs_attr *h, void *stream);

/* Estimate of the equi-join of the relations owning attributes u and v on u = v (u != v,
 * same component): per repetition the inner product of the two sketches (Eq. 5 with
 * r = 2), then the lower median; exact as int128 whenever sum_j |c_u c_v| < 2^126
 * (`exact`), else fp64.  reps: optional per-repetition detail.  Synchronous on stream.
 * Errors: CS_EINVAL (attributes out of range, equal, or in different components). */
cs_status cs_attr_estimate_join(cs_attr *h, int32_t u, int32_t v, void *stream, cs_estimate_t *out,
                                const cs_reps_t *reps);

/* Copy attribute u's counters, int64 [d][m], to host memory (synchronises the device). */
cs_status cs_attr_read(const cs_attr *h, int32_t u, int64_t *host_out);

/* Copy the hash coefficients: sign [d][n_comp][4], bin [d][n_comp][2] (either may be NULL). */
cs_status cs_attr_coefficients(const cs_attr *h, uint64_t *sign_out, uint64_t *bin_out);

/* ------------------------------------------------------------------ sub-query sketches */

/* Sketches of the sub-queries a query optimizer evaluates (Sec. 3.4), built in one pass
 * over each relation.  A sub-query is a connected set of the base query's joins, given
 * as a bit mask (bit e = join e of `graph`); it is the query on the relations those
 * joins touch, renumbered in ascending base order (relations, then attributes that one
 * of its joins names, then its joins).
 *
 * Hash functions (drawn from SplitMix64(seed), each coefficient its output >> 3,
 * redrawn when equal to p = 2^61 - 1): first, for each repetition t and base component
 * q, a shared sign polynomial a0..a3 and a bin polynomial b0, b1 (the order and values
 * cs_attr_create draws); then, for each repetition t and join e, a sign polynomial
 * a0..a3.  In a sub-query, an attribute's bin hash is its base component's; a join's
 * sign hash is its component's shared polynomial when it is the only join of that
 * component in the sub-query (so an attribute's sketch is reused by every sub-query
 * that joins it once, e.g. a pairwise join), and the join's own polynomial when the
 * component holds two or more of the sub-query's joins (an attribute joined twice needs
 * independent signs).  A relation's sketch in a sub-query is then fixed by its joined
 * columns and their sign polynomials; the distinct sketches ("targets", int64 [d][m]
 * each) are kept once and every sub-query reads its relations' targets.
 *
 * cs_subq_create: 2 <= m <= 2^20 (any m), 1 <= d <= 64, 1 <= n_sub <= 4096 masks,
 *   relations of at most 4 attributes, at most 16 targets and 16 distinct (column, sign
 *   polynomial) pairs per relation; allocates the targets' counters and a pass-1
 *   buffer of at most ~256 MB.  Errors: CS_EINVAL (a mask that is empty, names no join
 *   of the graph or is not connected; limits), CS_EGRAPH, CS_ENOMEM, CS_EDEVICE.
 * cs_subq_update: one pass over n tuples of base relation rel (keys uint32 [n][a_rel]
 *   as cs_update takes them, weights int64 [n] or NULL; device or pinned memory) adds
 *   every target of rel (Alg. 2 with each target's columns and hash functions).
 *   Deltas +1 (NULL) or +-1 with CS_UPDATE_UNIT_WEIGHTS take the two-pass record path;
 *   other weights one global atomic per (tuple, target, repetition).  Stream-ordered,
 *   allocates nothing; calls on one handle must not overlap (they share the pass-1
 *   buffer).
 * cs_subq_reset: zero every counter (stream-ordered).
 * cs_subq_estimate: the estimate of sub-query q (Eq. 5 / Alg. 3 as cs_estimate, with
 *   its plan), synchronous on stream; reps optional as for cs_estimate.
 * cs_subq_estimate_all: every sub-query's estimate in one batched estimate (outs[n_sub]).
 * cs_subq_layout: *n_targets, and target_of [n_sub][n_rel] = the target holding base
 *   relation k's sketch in sub-query q (-1 when k is not in q); either may be NULL.
 * cs_subq_read: copy target i's counters, int64 [d][m], to host memory (synchronises).
 * cs_subq_coefficients: comp_sign [d][Q][4], bin [d][Q][2], join_sign [d][E][4] (any
 *   may be NULL). */
typedef struct cs_subq cs_subq;  /* opaque */
cs_status cs_subq_create(const cs_graph *graph, const uint32_t *sub_joins, int32_t n_sub, uint32_t m,
                         uint32_t d, uint64_t seed, cs_subq **out);
cs_status cs_subq_destroy(cs_subq *h);
cs_status cs_subq_update(cs_subq *h, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                         int32_t flags, void *stream);
cs_status cs_subq_reset(cs_subq *h, void *stream);
cs_status cs_subq_estimate(cs_subq *h, int32_t q, void *stream, cs_estimate_t *out, const cs_reps_t *reps);
cs_status cs_subq_estimate_all(cs_subq *h, void *stream, cs_estimate_t *outs);
cs_status cs_subq_layout(const cs_subq *h, int32_t *n_targets, int32_t *target_of);
cs_status cs_subq_read(const cs_subq *h, int32_t target, int64_t *host_out);
cs_status cs_subq_coefficients(const cs_subq *h, uint64_t *comp_sign, uint64_t *bin, uint64_t *join_sign);

/* ------------------------------------------------------------------ AMS multi-join baseline */

/* The AMS multi-join sketch of Eq. 1 (Dobra et al.; Sec. 2), the method the convolution
 * sketch is measured against (Sec. 4): counter j of repetition t of relation R_k is
 *   c_{k,t,j} = sum_i Delta_i prod_{u in Omega(R_k)} prod_{v in Gamma(u)} s_{t,j,{u,v}}(i_u),
 * with its own degree-3 sign polynomial per join for every (t, j), drawn from the seeded
 * SplitMix64 stream (each draw >> 3, redrawn when equal to 2^61 - 1) in the order t, j,
 * join, a0..a3.  An update touches all d x m counters of the relation, O(d m) per tuple
 * against the Count sketch's O(d).  The estimate of repetition t is
 * X_t = (1/m) sum_j prod_k c_{k,t,j} (Thm. 2.3); the result is the lower median over t. */
typedef struct cs_ams cs_ams;  /* opaque */

typedef struct cs_ams_estimate_t {
    double value;            /* median X_t (fp64 of the exact numerator / m when exact) */
    int64_t num_lo, num_hi;  /* exact numerator S = m X of that repetition, two's
                                complement int128 (when exact = 1) */
    int32_t exact;           /* 1: every repetition's numerator is exact (|S_t| < 2^126) */
    int32_t median_rep;      /* repetition the median comes from */
} cs_ams_estimate_t;

/* Validate the graph (as cs_create; every relation must have 1 to 8 joins), draw the
 * coefficients, allocate r*d*m int64 counters on the current device and zero them.
 * 1 <= m <= 2^20, 1 <= d <= 64.  Errors: CS_EINVAL, CS_EGRAPH, CS_ENOMEM, CS_EDEVICE. */
cs_status cs_ams_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, cs_ams **out);

/* Free the handle (synchronises the device first). */
cs_status cs_ams_destroy(cs_ams *h);

/* Add n tuples to relation rel: keys uint32 [n][a_rel] tuple-major (device), weights
 * int64 [n] (device) or NULL for Delta = +1.  Stream-ordered; counters wrap mod 2^64. */
cs_status cs_ams_update(cs_ams *h, int32_t rel, const uint32_t *keys, const int64_t *weights,
                        uint64_t n, void *stream);

/* Zero every counter (stream-ordered). */
cs_status cs_ams_reset(cs_ams *h, void *stream);

/* Estimate (synchronous on `stream`).  rep_lo / rep_hi / rep_exact: optional host arrays
 * of d entries receiving each repetition's numerator S_t (wrapping int128 halves; exact
 * where rep_exact is 1). */
cs_status cs_ams_estimate(cs_ams *h, void *stream, cs_ams_estimate_t *out, int64_t *rep_lo,
                          int64_t *rep_hi, int32_t *rep_exact);

/* Copy relation rel's counters, int64 [d][m], to host memory (synchronises the device). */
cs_status cs_ams_read(const cs_ams *h, int32_t rel, int64_t *host_out);

/* Copy the sign coefficients, uint64 [d][m][n_edge][4], to host memory. */
cs_status cs_ams_coefficients(const cs_ams *h, uint64_t *host_out);

#ifdef __cplusplus
}
#endif

#endif /* CSKETCH_H */
