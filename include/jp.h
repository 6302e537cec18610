/*
 * jp.h -- C ABI of the MI355X (gfx950) Join-Project library.
 *
 * Operation (paper Sec. 1, Eq. 1): given R(x, y) and S(z, y), return the set
 *   PI_{x,z}( R JOIN_y S ) = { (x, z) : some y has (x, y) in R and (z, y) in S }.
 * The method (paper Sec. 2, Alg. 1): map x, y, z values to dense ids (Sec. 2.2,
 * with the semi-join on y of optimisation 2), build CSR for R, split S by z into
 * a sparse and a dense part (intersection-free partition, Sec. 2.3), compute
 * the sparse part with SparseBMM (Sec. 2.4, Alg. 2) and the dense part with
 * DenseEC (Sec. 2.5, Alg. 3), and return the disjoint union.
 *
 * Conventions for every call:
 *  - Column arguments are int32 DEVICE pointers (HIP device memory); any int32
 *    value is allowed, including negatives and INT32_MIN/INT32_MAX.  Input
 *    tuples may repeat; the result is a set (repeats never change it).
 *  - Work is enqueued on the caller's stream.  A call synchronises that stream
 *    only where noted ("syncs").  No call synchronises the device.
 *  - Every call returns a jp_status and never throws.  On failure
 *    jp_last_error() returns a message (thread-local, valid until the next call
 *    on the same thread).  Argument checks happen before any device work.
 *  - Output pairs are ORIGINAL values, ordered by (x, z) as signed int32, so
 *    consecutive chunks of a materialised result concatenate to the full list.
 *  - Counts are int64.  Per plan, each input side holds at most 2^31 - 1 tuples.
 *  - A plan or batch object is not thread-safe; distinct objects may be used
 *    concurrently from different threads on different streams.
 */
#ifndef JP_H_
#define JP_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JP_OK = 0,
  JP_EINVAL = 1,  /* bad argument (null pointer with n > 0, n < 0, n > 2^31-1, bad option) */
  JP_ENOMEM = 2,  /* device allocation failed or workspace_limit_bytes exceeded */
  JP_EHIP = 3,    /* a HIP runtime call failed; jp_last_error() has its text */
  JP_ESTATE = 4,  /* call out of order (e.g. count before execute) */
  JP_ERANGE = 5,  /* first > number of pairs in the requested part */
  JP_EBUSY = 6    /* server queue full or budget exhausted */
} jp_status;

/* Which part of the result: the union, or one side of the partition by z. */
typedef enum { JP_PART_ALL = 0, JP_PART_DENSE = 1, JP_PART_SPARSE = 2 } jp_part;

/* How the dense/sparse threshold tau is chosen (Sec. 2.6, function f2). */
typedef enum {
  JP_TAU_AUTO = 0,  /* cost model: z is dense iff m_z > tau, tau from f2 with GPU constants */
  JP_TAU_FIXED = 1  /* use jp_options.dense_threshold */
} jp_tau_mode;

/* Kernel of the DenseEC count pass (Sec. 2.5).  The write pass of
 * jp_materialize always uses the bit path; both are exact. */
typedef enum {
  JP_DENSE_AUTO = 0, /* the INT8-MFMA product for a single-query plan whose (x, dense key) panel has at
                        least 1/32 of its cells set and fits (2 GiB per panel); the bit path otherwise */
  JP_DENSE_BITS = 1, /* bit rows of the hot join keys ORed per window, cold keys scattered */
  JP_DENSE_MFMA = 2  /* 0/1 product on the INT8 matrix cores with int32 sums tested > 0, whenever the
                        plan is a single query and the panels fit; the bit path otherwise */
} jp_dense_kernel;

/* Evaluation path of a plan (paper Sec. 2.6, f1, and Fig. 1): the hybrid DIM^3
 * path (mapping, partition, SparseBMM + DenseEC) or the classical solution of
 * Sec. 1.1 (hash join, then deduplication of the projected join rows in a
 * device hash set; no mapping).  JP_STRATEGY_AUTO takes the classical path when
 * f1 > 0, i.e. when the join rows it must deduplicate cost less than the
 * mapping it avoids: OUT_J < ratio * (|R| + |S|), with OUT_J estimated from up
 * to 4096 sampled tuples per side (exact for smaller inputs).  AUTO considers
 * the classical path only with tau_mode AUTO, dense_kernel AUTO and no
 * JP_FLAG_GRAPH.  The classical path takes at most 2^30 join rows (JP_EINVAL
 * when forced beyond; AUTO then runs the hybrid path).  Its result has no dense
 * part (every pair is in JP_PART_SPARSE) and jp_plan_work reports zeros. */
typedef enum {
  JP_STRATEGY_AUTO = 0,
  JP_STRATEGY_HYBRID = 1,
  JP_STRATEGY_CLASSICAL = 2
} jp_strategy;

/* jp_options.flags bits */
#define JP_FLAG_TIMING 1 /* record HIP events around the kernels of jp_execute (see jp_plan_timings) */
#define JP_FLAG_GRAPH 2  /* record the count pass of the second jp_execute into a HIP graph and
                            replay it on later calls: no allocation and one launch per call after
                            the first; results are identical; JP_FLAG_TIMING is ignored with it */
#define JP_FLAG_DIRECT_IDS 4 /* columns whose values fill a dense range skip the sort that maps x and
                                z to ids (Sec. 2.2, optimisation 1: values already natural numbers):
                                ids, counts and the grouping come from a histogram over the key space,
                                scans and a scatter with per-key cursors.  Results are identical; on
                                gfx950 its per-element global atomics make it slower than the
                                default radix-sort mapping, so it is opt-in */

/* Options; an all-zero struct (or NULL) selects every default. */
typedef struct {
  int32_t tau_mode;              /* jp_tau_mode */
  int32_t dense_kernel;          /* jp_dense_kernel */
  int64_t dense_threshold;       /* JP_TAU_FIXED: z dense iff m_z > value (-1: all dense, INT64_MAX: none) */
  int32_t k_hot_max;             /* cap on hot join keys per instance in DenseEC (0 = 256; max 1024) */
  int32_t flags;                 /* JP_FLAG_* bits; others must be 0 */
  int64_t workspace_limit_bytes; /* 0 = no limit; else the most device memory the plan or batch may hold
                                    at once, temporaries included: exceeding it returns JP_ENOMEM */
  int32_t window_group;          /* z windows per workgroup of the bit-path DenseEC count (0 = automatic, max 64) */
  int32_t strategy;              /* a jp_strategy value, for plans: batches, servers, jp_tune and
                                    jp_count_static run the hybrid path and reject JP_STRATEGY_CLASSICAL */
  int32_t sparse_light_max;      /* SparseBMM count: rows with at most this much work run one per wavefront
                                    (0 = tuned or 1024; max 1024); heavier rows take a workgroup */
  int32_t sparse_med_max;        /* SparseBMM count: rows up to this much work run one per workgroup with one
                                    LDS hash set, heavier ones per z window (0 = tuned or 8192; at least
                                    sparse_light_max, max 8192) */
  int32_t mfma_tile;             /* tile of the INT8-MFMA product: 0 = tuned or 256 x 256, 1 = 128 x 256,
                                    2 = 256 x 128 (rows x dense z per workgroup) */
  int32_t reserved;              /* must be 0 */
} jp_options;

/* Kernel times of the last jp_execute (filled by jp_plan_timings for a plan
 * built with JP_FLAG_TIMING) and the algorithmic work of those kernels (filled
 * by jp_plan_work), for roofline accounting. */
typedef struct {
  float sparse_ms;            /* SparseBMM count kernels */
  float dense_ms;             /* DenseEC count kernel */
  float execute_ms;           /* all of jp_execute */
  float pad_;
  int64_t sparse_join_rows;   /* sum over x of |S_sparse[y]| for y in R[x] (join rows reaching sparse z) */
  int64_t n_r_kept;           /* R tuples after the semi-join (CSR entries read) */
  int64_t n_x;                /* x rows */
  int64_t dense_hot_words;    /* sum over x of (hot keys of x) * (32-bit words of its dense z range) */
  int64_t dense_row_words;    /* sum over x of the words of its dense z range (one popcount each) */
  int64_t dense_cold_entries; /* cold dense S entries scattered, summed over x */
  int64_t dense_mfma_ops;     /* 2 * |X| * (dense keys) * |Z_dense| when the INT8-MFMA product ran, else 0 */
  float map_ms;               /* plan: input gather and mapping to ids with the CSR builds (Sec. 2.2) */
  float partition_ms;         /* plan: partition by z and the DenseEC tables (Sec. 2.3) */
  int64_t dense_mfma_issued_ops; /* int8 ops the INT8-MFMA product issued (padded tiles, up to each tile's
                                    early stop), else 0 */
} jp_timings;

typedef struct {
  int64_t n_x, n_y, n_z;   /* distinct x (after the semi-join), y (of S), z */
  int64_t n_r_kept;        /* R tuples whose y occurs in S (semi-join, Sec. 2.2 opt. 2) */
  int64_t out_j;           /* bag join size: sum over y of d_R(y) * d_S(y) */
  int64_t tau;             /* threshold used: z dense iff m_z > tau */
  int64_t n_z_dense;       /* number of dense z */
  int64_t k_hot;           /* hot join keys held as bit rows in DenseEC */
  int64_t footprint_bytes; /* device memory owned by the object for this instance's share */
  int64_t pivot_cover;     /* dense z in the S row of the pivot key whose rows DenseEC counts outside
                              that row (0: no pivot split for this instance) */
  int64_t dense_mfma;      /* 1 if the dense part is counted by the INT8-MFMA product, else 0 */
  int64_t peak_bytes;      /* most device memory the object held at once so far, temporaries included
                              (all instances of a batch; the quantity workspace_limit_bytes bounds) */
  int64_t map_direct;      /* bit 0: z ids, bit 1: x ids came from the direct-range mapping (no sort) */
  int64_t strategy;        /* JP_STRATEGY_HYBRID or JP_STRATEGY_CLASSICAL: the path the plan runs */
} jp_stats;

typedef struct jp_plan jp_plan;
typedef struct jp_batch jp_batch;

/* ---------------------------------------------------------------- plan --- */

/* Build the mapped, partitioned plan of one query (Alg. 1 up to the kernels:
 * mapping, CSR of R, partition of S by z).  r_x/r_y hold n_r tuples of R and
 * s_z/s_y hold n_s tuples of S, all device pointers that must stay valid until
 * the work enqueued by this call has completed.  Syncs `stream` (to size the
 * plan).  On success *out owns all device memory it uses. */
jp_status jp_plan_create(const int32_t* r_x, const int32_t* r_y, int64_t n_r,
                         const int32_t* s_z, const int32_t* s_y, int64_t n_s,
                         const jp_options* opt, hipStream_t stream, jp_plan** out);

/* Count pass of SparseBMM (Alg. 2) and DenseEC (Alg. 3) for every x row, and
 * the per-row offsets of the result.  Asynchronous. */
jp_status jp_execute(jp_plan* p, hipStream_t stream);

/* Host copies of the number of pairs in the union, the dense and the sparse
 * part (each output nullable).  JP_ESTATE before jp_execute.  Syncs. */
jp_status jp_count(jp_plan* p, int64_t* total, int64_t* dense, int64_t* sparse,
                   hipStream_t stream);

/* Write pairs [first, first + max_pairs) of the sorted result of `part` into
 * the device buffers out_x / out_z (caller-owned, >= max_pairs int32 each).
 * *n_written (host) receives min(max_pairs, count - first).  first == count
 * writes nothing and returns JP_OK; first > count returns JP_ERANGE.  Syncs. */
jp_status jp_materialize(jp_plan* p, jp_part part, int64_t first, int64_t max_pairs,
                         int32_t* out_x, int32_t* out_z, int64_t* n_written,
                         hipStream_t stream);

/* Host copies of the distinct x values (n_x entries, ascending) and of the
 * per-row offsets of `part` in the sorted result (n_x + 1 entries); rows can
 * then be materialised one at a time.  Either output may be NULL.  Syncs. */
jp_status jp_row_info(jp_plan* p, jp_part part, int32_t* x_values, int64_t* row_offsets,
                      hipStream_t stream);

/* Host copy of the dense z values (n_z_dense entries, ascending).  Syncs. */
jp_status jp_dense_z(jp_plan* p, int32_t* z_values, hipStream_t stream);

jp_status jp_plan_stats(const jp_plan* p, jp_stats* s);

/* Kernel times of the last jp_execute, and of the mapping and partition
 * stages of the plan, into the *_ms fields (others zeroed); JP_ESTATE unless
 * the plan was created with JP_FLAG_TIMING and executed.  Syncs. */
jp_status jp_plan_timings(jp_plan* p, jp_timings* t, hipStream_t stream);

/* Algorithmic work counters of the execute kernels into the integer fields of
 * *t (the *_ms fields are left as they are); JP_ESTATE before jp_execute.
 * Runs one small kernel.  Syncs. */
jp_status jp_plan_work(jp_plan* p, jp_timings* t, hipStream_t stream);
void jp_plan_destroy(jp_plan* p); /* NULL-safe; frees all plan-owned device memory */

const char* jp_last_error(void);

/* ------------------------------------------------- no device allocation --- */

/* Size of the static device scratch of jp_count_static, and the most tuples
 * (n_r + n_s) it accepts. */
#define JP_STATIC_SCRATCH_MIB 256
#define JP_STATIC_MAX_TUPLES (1 << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same result as jp_plan_create +
 * jp_execute + jp_count on one query, computed entirely inside a fixed
 * device array of JP_STATIC_SCRATCH_MIB MiB that the library holds per GPU
 * until the process ends; the call allocates and frees no device memory.
 * Columns as for jp_plan_create; counts go to host outputs (each nullable).
 * JP_EINVAL (before any device work) if n_r + n_s > JP_STATIC_MAX_TUPLES or
 * the options ask for JP_FLAG_TIMING or JP_FLAG_GRAPH; JP_ENOMEM if the
 * query's plan does not fit the scratch (very wide value domains).  Syncs.
 * Calls from threads of one process are serialised per GPU (the array is the
 * process's own); work of an earlier call never overlaps a later one, and
 * every call initialises the parts of the array it reads. */
jp_status jp_count_static(const int32_t* r_x, const int32_t* r_y, int64_t n_r,
                          const int32_t* s_z, const int32_t* s_y, int64_t n_s,
                          const jp_options* opt, hipStream_t stream,
                          int64_t* total, int64_t* dense, int64_t* sparse);

/* --------------------------------------------------------------- batch --- */

/* One query of a batch: device columns as for jp_plan_create. */
typedef struct {
  const int32_t* r_x;
  const int32_t* r_y;
  const int32_t* s_z;
  const int32_t* s_y;
  int64_t n_r;
  int64_t n_s;
} jp_instance;

/* Many independent queries planned together: every stage runs as one launch
 * over all instances (block-diagonal id spaces), with tau and the hot key set
 * chosen per instance.  The array `inst` is read during the call (host
 * memory); its device columns must stay valid until the enqueued work has
 * completed.  The sum of tuples per side must stay below 2^31.  Syncs. */
jp_status jp_batch_create(const jp_instance* inst, int32_t n_inst, const jp_options* opt,
                          hipStream_t stream, jp_batch** out);
jp_status jp_batch_execute(jp_batch* b, hipStream_t stream);
/* Per-instance pair counts into host array totals[n_inst].  Syncs. */
jp_status jp_batch_counts(jp_batch* b, int64_t* totals, hipStream_t stream);
jp_status jp_batch_materialize(jp_batch* b, int32_t inst, jp_part part, int64_t first,
                               int64_t max_pairs, int32_t* out_x, int32_t* out_z,
                               int64_t* n_written, hipStream_t stream);
jp_status jp_batch_stats(const jp_batch* b, int32_t inst, jp_stats* s);
/* As jp_plan_timings and jp_plan_work, over all instances of the batch. */
jp_status jp_batch_timings(jp_batch* b, jp_timings* t, hipStream_t stream);
jp_status jp_batch_work(jp_batch* b, jp_timings* t, hipStream_t stream);
void jp_batch_destroy(jp_batch* b);

/* ------------------------------------------------------------ autotuner --- */

/* The dense/sparse threshold of Sec. 2.6 is tau = (c_de / c_sp) |X| |S| / OUT_J;
 * jp_tune times the plan + count pass of one query (device columns as for
 * jp_plan_create) for a set of thresholds (all dense, all sparse, the model's
 * tau scaled by 1/16 .. 16, quantiles of m_z) in increasing order, skipping
 * the higher ones once a threshold above the best is 3x slower than it, checks
 * that all give the same counts (the partition is intersection-free, Sec.
 * 2.3), then, at the fastest
 * threshold, searches the DenseEC count kernel (bit path or INT8 MFMA), the
 * hot-key cap and the windows per workgroup one after the other (a setting
 * replaces the current best only when at least 2% faster).  The cost
 * ratio and these choices are stored under the query's shape signature (log2
 * buckets of |X|, |Z|, |S| and OUT_J / |S|); later plans and batch instances
 * of that signature use them for every option left automatic (tau_mode
 * JP_TAU_AUTO, dense_kernel JP_DENSE_AUTO, k_hot_max 0, window_group 0,
 * sparse_light_max 0, sparse_med_max 0, mfma_tile 0; batches take the
 * SparseBMM bounds and the tile from their first instance's record).  The
 * store is process-wide and thread-safe.  jp_tune syncs the stream; it returns
 * JP_ESTATE if two settings disagree on the counts. */
typedef struct {
  int64_t tau;         /* fastest threshold (dense iff m_z > tau; INT64_MAX: all sparse) */
  int64_t model_tau;   /* the untuned cost model's threshold */
  double cost_ratio;   /* c_de / c_sp stored for the signature */
  double best_ms;      /* plan + count pass at tau (best of 2) */
  double model_ms;     /* the same at model_tau */
  int32_t candidates;  /* settings timed besides the model's */
  int32_t dense_kernel;  /* chosen jp_dense_kernel */
  int32_t k_hot_max;     /* chosen hot-key cap */
  int32_t window_group;  /* chosen windows per workgroup */
  uint64_t signature;  /* shape signature the choices are stored under */
  int32_t sparse_light_max;  /* chosen SparseBMM one-wavefront-per-row bound */
  int32_t sparse_med_max;    /* chosen SparseBMM one-workgroup-per-row bound */
  int32_t mfma_tile;         /* chosen INT8-MFMA tile */
  int32_t pad_;
} jp_tune_result;

jp_status jp_tune(const int32_t* r_x, const int32_t* r_y, int64_t n_r, const int32_t* s_z, const int32_t* s_y,
                  int64_t n_s, const jp_options* opt, hipStream_t stream, jp_tune_result* out);
jp_status jp_tune_clear(void); /* forgets every stored ratio */

/* -------------------------------------------------------------- server --- */

/* A query server: a host thread that admits submitted queries while their
 * estimated device footprint fits an HBM budget, plans every admitted group
 * as one batch (continuous batching: queries that arrive while a batch runs
 * join the next one) and overlaps the planning of one batch with the
 * execution of the previous one on a second stream.  The paper runs one query
 * at a time (Sec. 5); the server only groups independent queries, so each
 * result is exactly that of the query alone.
 *
 * Admission.  A query's estimated footprint is a fixed number of bytes per
 * input tuple (its plan, temporaries included) plus, with JP_SERVER_DIGEST or
 * JP_SERVER_KEEP, one chunk of output of min(n_r * n_s, chunk_pairs) pairs.
 * A group is admitted while the sum of the estimates of everything in flight
 * or kept stays within hbm_budget_bytes and each side of the group holds at
 * most 2^31 - 1 tuples; the group's plan is then limited to its summed
 * estimate (every device byte it holds at once), so the server never holds
 * more than the budget (the caching allocator may keep freed blocks).  A
 * query whose estimate exceeds the budget fails with JP_ENOMEM.  A group
 * whose plan fails is split in halves and planned again, so a failure stays
 * with the query that causes it: a query above its estimate is retried once
 * alone with all the budget left, and fails with JP_ENOMEM if that is no
 * more.  Results: counts, the order-independent digest (JP_SERVER_DIGEST:
 * the wrapping sum of SplitMix64(key(x, z)) over the pairs, key = the two
 * sign-flipped values with x in the high word, computed on the device from
 * materialised chunks) and, with JP_SERVER_KEEP, the pairs themselves until
 * the query is released. */
typedef struct jp_server jp_server;

#define JP_SERVER_DIGEST 1 /* compute each query's digest on the device before it is done */
#define JP_SERVER_KEEP 2   /* keep each query's plan until jp_server_release: jp_server_materialize */

typedef struct {
  int32_t device;           /* HIP device the server runs on */
  int32_t max_batch;        /* most queries per batch (0 = 4096) */
  int64_t hbm_budget_bytes; /* device memory the in-flight and kept batches may hold (0 = 64 GiB) */
  jp_options opt;           /* options of every batch (no JP_FLAG_TIMING / JP_FLAG_GRAPH) */
  int32_t flags;            /* JP_SERVER_* bits */
  int32_t reserved;         /* must be 0 */
  int64_t chunk_pairs;      /* pairs per output chunk of the digest pass and the estimate (0 = 2^24) */
} jp_server_config;

typedef struct {
  int64_t total, dense, sparse; /* pair counts */
  uint64_t digest;              /* digest of the pairs when has_digest */
  int32_t status;               /* jp_status of the query */
  int32_t batch_size;           /* queries in the batch that carried it */
  int32_t has_digest;           /* 1 if digest is set (JP_SERVER_DIGEST) */
  int32_t kept;                 /* 1 while the pairs can be materialised (JP_SERVER_KEEP, not released) */
  double submit_us, admit_us, done_us; /* host clock, microseconds since the server started */
} jp_query_result;

typedef struct {
  int64_t submitted, completed, failed, batches;
  int64_t splits;          /* failed groups split in halves and planned again */
  int64_t pairs;           /* pairs over completed queries */
  int64_t peak_bytes;      /* largest sum of the live batches' peak device bytes (<= budget_bytes) */
  int64_t budget_bytes;    /* the HBM budget */
  int64_t charged_bytes;   /* estimates of the batches live now (in flight or kept) */
  double p50_us, p99_us, mean_us; /* latency submit -> done over completed queries */
} jp_server_summary;

/* Starts the server thread.  Syncs nothing on the caller's streams.
 * JP_EINVAL for a bad device, negative limits, unknown flags or options. */
jp_status jp_server_create(const jp_server_config* cfg, jp_server** out);

/* Queues one query.  q holds device columns as in jp_plan_create; they must
 * stay valid until the query is done.  JP_EBUSY if the server is stopping. */
jp_status jp_server_submit(jp_server* s, const jp_instance* q, uint64_t* ticket);

/* *done = 1 and *r filled once the query has finished; non-blocking. */
jp_status jp_server_poll(jp_server* s, uint64_t ticket, int* done, jp_query_result* r);

/* Blocks until the query has finished, then fills *r. */
jp_status jp_server_wait(jp_server* s, uint64_t ticket, jp_query_result* r);

/* As jp_materialize, for a finished query of a JP_SERVER_KEEP server that has
 * not been released (else JP_ESTATE).  Requests of up to chunk_pairs pairs fit
 * the query's admission estimate; larger ones may return JP_ENOMEM.  Runs on
 * the caller's stream; syncs it. */
jp_status jp_server_materialize(jp_server* s, uint64_t ticket, jp_part part, int64_t first,
                                int64_t max_pairs, int32_t* out_x, int32_t* out_z,
                                int64_t* n_written, hipStream_t stream);

/* Drops a finished query's kept result; its batch's memory and budget charge
 * go once every kept query of the batch is released.  JP_ESTATE if not done. */
jp_status jp_server_release(jp_server* s, uint64_t ticket);

jp_status jp_server_stats(jp_server* s, jp_server_summary* st);

/* Finishes the queued queries, stops the thread, frees everything, kept
 * results included (NULL-safe). */
void jp_server_destroy(jp_server* s);

/* ------------------------------------------------ partial result cache --- */

/* Partial result caching (paper Sec. 3).  The result splits by z (the
 * intersection-free partition), so the results of a subset Z_cached of the z
 * values can be kept: a later run on the same tables omits the S tuples whose
 * z is cached (jp_plan_create_cached), and its result together with the
 * cached pairs (jp_cache_materialize) is the full result; the two parts are
 * disjoint and their counts add.
 *
 * jp_cache_build ranks the z of an executed single-query hybrid plan by
 * CacheScore(z) = cost(z) / space(z) and caches, in that order, those whose
 * space fits budget_bytes (4 bytes a word):
 *   cost(z)  = OUT_{J,z} (join rows reaching z) for a sparse z, and
 *              (c_de / c_sp) * |X| for a dense z (the partition's cost model);
 *   space(z) = 2 + min(k, |X| - k) words, k = number of x with (x, z) in the
 *              result: the x list, or its complement in X when k > |X| / 2.
 * Building reads the plan's result once (chunked, on the device).  JP_ESTATE if
 * the plan was not executed; JP_EINVAL for a batch or a classical plan.
 * Syncs.  The cache is valid for the tables it was built from; the caller
 * passes the same tables to jp_plan_create_cached (whose sizes it checks). */
typedef struct jp_cache jp_cache;
jp_status jp_cache_build(jp_plan* p, int64_t budget_bytes, hipStream_t stream, jp_cache** out);
/* Cached z values, cached pairs and words of storage (host outputs, nullable). */
jp_status jp_cache_info(const jp_cache* c, int64_t* n_z, int64_t* pairs, int64_t* words);
/* The cached z values, ascending (host array of n_z). */
jp_status jp_cache_z(const jp_cache* c, int32_t* z_values);
/* A plan over R and the S tuples whose z is not cached (arguments as for
 * jp_plan_create).  Syncs. */
jp_status jp_plan_create_cached(const int32_t* r_x, const int32_t* r_y, int64_t n_r, const int32_t* s_z,
                                const int32_t* s_y, int64_t n_s, const jp_cache* c, const jp_options* opt,
                                hipStream_t stream, jp_plan** out);
/* Cached pairs [first, first + max_pairs) sorted by (z, x) as signed int32,
 * into caller device buffers; first == pairs writes nothing, first > pairs is
 * JP_ERANGE.  Syncs. */
jp_status jp_cache_materialize(const jp_cache* c, int64_t first, int64_t max_pairs, int32_t* out_x, int32_t* out_z,
                               int64_t* n_written, hipStream_t stream);
/* Frees the cache (NULL-safe). */
void jp_cache_destroy(jp_cache* c);

/* ---------------------------------------------------- Join-Aggregate --- */

/* Join-Aggregate with group-by attributes from both tables (paper Sec. 4.1):
 *   G_{x,z} COUNT(*), SUM(R.v * S.u)  over  R(x, y, v) JOIN_y S(z, y, u).
 * The groups are the Join-Project result (the same (x, z) set); each carries
 * the number of its join rows (repeated tuples count) and the sum of v * u over
 * them as int64 (wrapping on overflow).  As the paper adapts DIM^3, the
 * deduplicating accumulator of each x row becomes an aggregate accumulator:
 * rows with little work aggregate in an LDS hash map, heavier rows in dense
 * LDS accumulators over windows of z.  Columns are int32 device arrays, read
 * only during jp_agg_create.  Errors as for jp_plan_create.  Syncs. */
typedef struct jp_agg jp_agg;
jp_status jp_agg_create(const int32_t* r_x, const int32_t* r_y, const int32_t* r_v, int64_t n_r,
                        const int32_t* s_z, const int32_t* s_y, const int32_t* s_u, int64_t n_s,
                        hipStream_t stream, jp_agg** out);
/* Count pass (number of groups per x row); asynchronous. */
jp_status jp_agg_execute(jp_agg* a, hipStream_t stream);
/* Number of groups and of join rows (host outputs, nullable).  JP_ESTATE
 * before jp_agg_execute.  Syncs. */
jp_status jp_agg_count(jp_agg* a, int64_t* groups, int64_t* out_j, hipStream_t stream);
/* Groups [first, first + max_groups) in (x, z) order (signed int32) into
 * caller device buffers: x and z values, counts and sums (int64).  As
 * jp_materialize: first == groups writes nothing, first > groups is JP_ERANGE.
 * Syncs. */
jp_status jp_agg_materialize(jp_agg* a, int64_t first, int64_t max_groups, int32_t* out_x, int32_t* out_z,
                             int64_t* out_count, int64_t* out_sum, int64_t* n_written, hipStream_t stream);
/* Frees the aggregate (NULL-safe). */
void jp_agg_destroy(jp_agg* a);

/* ---------------------------------------------------- composite keys --- */

/* Dictionary encoding of multi-attribute keys (paper Sec. 2.2, "Supporting
 * Wider Range of Join-Project Operations"): a tuple of columns is mapped to
 * one consecutive natural number, so a Join-Project whose x, y or z is a
 * tuple of attributes runs as the single-column operation over the ids.  The
 * id of a tuple is its rank among the distinct tuples in lexicographic order
 * (each column compared as signed int32): id order is tuple order, so a result
 * sorted by ids is sorted by tuples.  Parts encoded together share one
 * dictionary (R.y and S.y must, for their ids to join).
 *
 * cols[p * n_cols + c] is device column c of part p, n[p] rows (n_cols in
 * [1, 8]); ids[p] (device, n[p] int32) receives part p's ids.  The columns are
 * read only during the call; the dictionary keeps its own copy of the distinct
 * tuples.  JP_EINVAL for bad counts or null pointers (checked before any device
 * work), or more than 2^31 - 1 rows over all parts.  Syncs. */
typedef struct jp_dict jp_dict;
jp_status jp_dict_create(int32_t n_cols, int32_t n_parts, const int32_t* const* cols, const int64_t* n,
                         int32_t* const* ids, hipStream_t stream, jp_dict** out);
/* Number of distinct tuples (ids are [0, n_distinct)). */
jp_status jp_dict_size(const jp_dict* d, int64_t* n_distinct);
/* cols_out[c][i] = column c of the tuple with id ids[i] (device arrays of n
 * int32).  JP_ERANGE if any id lies outside [0, n_distinct).  Syncs. */
jp_status jp_dict_decode(const jp_dict* d, const int32_t* ids, int64_t n, int32_t* const* cols_out,
                         hipStream_t stream);
/* Frees the dictionary (NULL-safe). */
void jp_dict_destroy(jp_dict* d);

/* -------------------------------------------------------------- digest --- */

/* *digest (one uint64 in DEVICE memory) += the order-independent digest of the
 * n pairs (x[i], z[i]) (device columns): the wrapping sum of SplitMix64
 * (Steele, Lea and Flood, OOPSLA 2014) of key(x, z), the sign-flipped values
 * with x in the high word.  Adding the digests of the chunks of a result gives
 * the digest of the result.  Asynchronous. */
jp_status jp_digest_pairs(const int32_t* x, const int32_t* z, int64_t n, uint64_t* digest,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* JP_H_ */
