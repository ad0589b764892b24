/*
 * fdbscan.h - C ABI of libfdbscan: tree-based DBSCAN for 2D/3D float32 points on
 * one AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2.1 of Prokopenko, Lebrun-Grandie, Arndt, "Fast tree-based
 * algorithms for DBSCAN for low-dimensional data on GPUs", ICPP 2023): given n
 * points X in d = 2 or 3 dimensions, eps > 0 and minPts >= 1,
 *   N_eps(x) = { y in X : dist(x, y) <= eps }   (x itself included),
 *   x is core  <=>  |N_eps(x)| >= minPts,
 *   clusters   = connected components of the core points under "within eps",
 *   border     = non-core point within eps of a core point,
 *   noise      = the rest.
 * The method (Sections 3.2, 4.1, 4.2): a linear BVH over the points (FDbscan)
 * or over dense grid cells plus the remaining points (FDbscan-DenseBox), an
 * early-exit core-point pass, then one fused traversal that merges clusters in
 * a lock-free union-find as neighbours are found, without storing them.
 *
 * Distance test: both algorithms decide "within eps" as
 *   s <= fl32(eps*eps),  s = (dx*dx + dy*dy) + dz*dz  in fp32,
 * each difference, product and sum rounded on its own (no fused multiply-add,
 * no flush of denormals). Labels are therefore exact, not approximate.
 *
 * Conventions for every call below:
 *   - pointers without an h_ prefix are device pointers on the handle's device;
 *     h_ pointers are host pointers;
 *   - every call is ordered on `stream` (a hipStream_t; NULL = the default
 *     stream) and returns without waiting for the GPU, except where noted;
 *   - the caller owns every buffer it passes; the library writes only to the
 *     outputs and the workspace;
 *   - no call aborts, exits or throws; errors are returned as fdb_status and
 *     leave the outputs untouched when detected before any launch;
 *   - a handle is used by one host thread at a time; a call that finds another
 *     thread inside a call on the same handle returns FDB_ERR_BUSY at once.
 */
#ifndef FDBSCAN_H
#define FDBSCAN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdb_handle fdb_handle;

typedef enum {
  FDB_OK = 0,
  FDB_ERR_INVALID = 1,   /* bad argument: dim, n, eps, minPts, NULL pointer, options */
  FDB_ERR_NOMEM = 2,     /* workspace too small, or the handle could not allocate one */
  FDB_ERR_HIP = 3,       /* a HIP runtime call failed */
  FDB_ERR_NONFINITE = 4, /* a coordinate is NaN or infinite (reported when the call waits) */
  FDB_ERR_INTERNAL = 5,  /* a kernel's own consistency check failed (reported when the call waits) */
  FDB_ERR_BUSY = 6,      /* another host thread is inside a call on the same handle */
  FDB_ERR_SCRATCH = 7    /* fdb_dbscan_noalloc: the input needs more than FDB_NOALLOC_SCRATCH_BYTES */
} fdb_status;

typedef enum {
  FDB_ALGO_FDBSCAN = 0,  /* LBVH over all points (Section 4.1) */
  FDB_ALGO_DENSEBOX = 1, /* LBVH over dense eps/sqrt(d) grid cells + other points (Section 4.2) */
  /* Choose per input (Sections 5-6 leave the choice to a rule of thumb). Measured
     here, DenseBox is never more than ~15% slower than FDbscan (sparse data with
     no dense cells) and up to 20x faster, and the share of points in dense cells
     does not predict the rare cases FDbscan wins; so the choice is DenseBox.
     Batches (fdb_dbscan_batched) run DenseBox. */
  FDB_ALGO_AUTO = 2
} fdb_algo;

typedef enum {
  /* Cluster ids 0..K-1 in increasing order of the smallest input index among each
     cluster's core points; a border point takes the smallest id among the
     clusters holding a core point within eps of it. Labels are a pure function of
     (points, eps, minPts), identical for both algorithms. */
  FDB_BORDER_CANONICAL = 0,
  /* The paper's rule (Section 3.2): a border point joins the first cluster whose
     compare-and-swap claims it. Core flags, noise and the core partition are as in
     canonical mode; the choice among eligible clusters depends on timing. */
  FDB_BORDER_FIRST = 1,
  /* DBSCAN* (Section 2.1 names it; Section 6 lists it as future work): border
     points are not cluster members, so every non-core point is noise (-1). The
     clusters, their ids and K are those of canonical mode. */
  FDB_BORDER_NONE = 2
} fdb_border;

/* Launch-shape parameters (leaf_size, block_size, tile) left at 0 take the
   handle's tuned value for the call's shape when fdb_tune has stored one (see
   fdb_tune), else the built-in default. None of them changes any label. */
typedef struct {
  int32_t algo;       /* fdb_algo */
  int32_t border;     /* fdb_border */
  int32_t leaf_size;  /* traversal: subtrees of <= leaf_size primitives are scanned linearly (1..1024);
                         0 = tuned or default (8) */
  int32_t block_size; /* threads per workgroup of the traversal kernels (64..1024, multiple of 64);
                         0 = tuned or default (128) */
  int32_t tile;       /* traversal tile of the wavefront packet walks: candidates loaded per step, one
                         per lane (8..64); 0 = tuned or default (64) */
  uint32_t flags;     /* FDB_FLAG_* bits */
} fdb_options;        /* all-zero = FDbscan, canonical labels, tuned or default launch shape */

enum {
  /* Record the call's whole launch sequence once as a HIP graph (per handle, keyed
     by every argument but the stream) and replay it on later calls with the same
     arguments: one graph launch instead of ~40 kernel launches. The graph holds
     the buffers' addresses, so it is replayed only for exactly the same pointers,
     sizes and parameters; anything else records a new one (the handle keeps the
     16 most recent). Results are those of the plain call. */
  FDB_FLAG_GRAPH = 1u,
  /* Debug: after the fused main phase, check the union-find forest it left
     (fdb_debug_forest states the invariants) and raise FDB_INFO_FOREST if any
     point breaks them. One extra pass over the labels; labels are unchanged. */
  FDB_FLAG_VALIDATE = 2u
};

/* Information bits, read with fdb_last_info(). */
enum {
  FDB_INFO_DENSEBOX_FALLBACK = 1u, /* DenseBox (or the automatic choice): the eps/sqrt(d) grid needs more
                                      cells per axis than 64-bit keys hold (eps tiny against the extent),
                                      so the cells were widened to fit; density is still decided by the
                                      exact guard, labels are exact, fewer cells come out dense. */
  FDB_INFO_NONFINITE = 2u,         /* a NaN or infinite coordinate was seen; labels are undefined */
  FDB_INFO_INTERNAL = 4u,          /* a kernel stopped a walk that broke its own bounds; labels undefined */
  FDB_INFO_BAD_PARAMS = 8u,        /* batch: some cloud's eps is not finite and > 0, or its minPts < 1;
                                      that cloud's labels are undefined */
  FDB_INFO_AUTO_FDBSCAN = 16u,     /* no longer raised: the automatic choice always runs DenseBox (a grid
                                      too wide for 64-bit keys raises FDB_INFO_DENSEBOX_FALLBACK) */
  FDB_INFO_FOREST = 32u            /* FDB_FLAG_VALIDATE: the union-find forest broke its invariants */
};

/* Create a handle bound to HIP device `device`. *out receives the handle. */
fdb_status fdb_create(fdb_handle** out, int device);

/* Release the handle and every buffer it allocated. NULL is ignored. */
void fdb_destroy(fdb_handle* h);

/* Workspace bytes fdb_dbscan needs for n points of dimension dim with options
   opt (NULL = defaults). Depends on (n, dim, algo) only, never on eps or minPts:
   memory is linear in n (Section 3.2). */
fdb_status fdb_workspace_bytes(int64_t n, int32_t dim, const fdb_options* opt, size_t* h_out);

/*
 * Cluster `n` points.
 *   points     [n][dim] float32, row-major (point i at points[i*dim .. i*dim+dim-1]).
 *   n          0 <= n < 2^30.
 *   dim        2 or 3.
 *   eps        finite, > 0; the library compares squared distances with fl32(eps*eps).
 *   min_pts    >= 1. minPts <= 2 skips the core-point pass (Algorithm 3's special case).
 *   opt        NULL = defaults.
 *   labels     [n] int32 out, in input order: -1 noise, else cluster id 0..K-1.
 *   is_core    [n] uint8 out (1 = core point), or NULL.
 *   h_num_clusters  host int32 out (K), or NULL. When non-NULL the call waits for
 *              the stream, and returns FDB_ERR_NONFINITE if a coordinate was not finite
 *              (FDB_ERR_INTERNAL if a kernel's consistency check failed).
 *   workspace  device buffer of >= fdb_workspace_bytes() bytes, or NULL: then the
 *              handle allocates (and keeps, growing it when needed) its own.
 *   stream     hipStream_t the work is ordered on.
 * With h_num_clusters = NULL nothing waits for the GPU, for either algorithm
 * (DenseBox sizes its grid on the device), so the call can be recorded into a
 * HIP graph by stream capture; errors found on the device are then read with
 * fdb_last_status. The workspace is the caller's (or, when NULL, the handle's):
 * too small a caller workspace gives FDB_ERR_NOMEM before any launch.
 */
fdb_status fdb_dbscan(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                      const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                      void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Size of the library's static device scratch that fdb_dbscan_noalloc works in
   (one copy per GPU the library runs on, held until the process ends). */
#define FDB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * fdb_dbscan without any allocation, for callers that cannot allocate device or
 * host memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Arguments, results and errors are those of fdb_dbscan with
 * workspace = NULL, except:
 *   - the workspace is the library's static scratch of FDB_NOALLOC_SCRATCH_BYTES
 *     on the handle's device (no hipMalloc, no hipFree, no allocating library
 *     call; the handle was set up by fdb_create). An input whose
 *     fdb_workspace_bytes exceeds it returns FDB_ERR_SCRATCH before any launch
 *     (64 MiB holds about 298k 3D points for DenseBox, 543k for FDbscan);
 *   - opt->flags must not hold FDB_FLAG_GRAPH (recording a graph allocates):
 *     FDB_ERR_INVALID;
 *   - stage timing (fdb_set_timing) is not recorded.
 * Every call on one GPU, from any handle, shares that GPU's scratch, which keeps
 * the last call's contents (each call clears what it needs): calls that overlap on
 * one GPU (other streams, other host threads with other handles) race and give
 * undefined labels. Order them on one stream or serialise them.
 */
fdb_status fdb_dbscan_noalloc(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                              const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                              hipStream_t stream);

/*
 * Cluster a batch of independent point clouds in one launch sequence (every
 * stage is one kernel launch for the whole batch; nothing waits for the GPU).
 * Cloud c is points[offsets[c] .. offsets[c+1]) (row-major [*][dim] float32, as
 * in fdb_dbscan) and is clustered on its own with eps[c] and min_pts[c]; its
 * labels (in input order, at the same positions) and is_core flags are exactly
 * what fdb_dbscan would give for that cloud alone, and num_clusters[c] its K.
 *   n_total       offsets[num_clouds]; 0 <= n_total < 2^30 (host value).
 *   offsets       device int64 [num_clouds+1], nondecreasing, offsets[0] = 0,
 *                 offsets[num_clouds] = n_total. Offsets outside [0, n_total] are
 *                 clamped (never read out of bounds) and raise FDB_INFO_BAD_PARAMS.
 *   num_clouds    1 .. 2^24.
 *   eps, min_pts  device float32 / int32 [num_clouds]; a cloud with eps not finite
 *                 and > 0, or min_pts < 1, raises FDB_INFO_BAD_PARAMS.
 *   labels        device int32 [n_total] out; is_core device uint8 [n_total] or NULL.
 *   num_clusters  device int32 [num_clouds] out, or NULL: K of each cloud, or -1
 *                 where that cloud's labels are undefined (a coordinate that is not
 *                 finite, bad eps/min_pts, or offsets out of order); other clouds'
 *                 results stay exact.
 *   workspace     >= fdb_workspace_bytes_batched() bytes, or NULL (handle-owned).
 * The core pass runs for every cloud (also minPts <= 2: same result). The
 * batch-wide error bits (FDB_INFO_NONFINITE, FDB_INFO_BAD_PARAMS,
 * FDB_INFO_INTERNAL) are read with fdb_last_info().
 */
fdb_status fdb_workspace_bytes_batched(int64_t n_total, int32_t num_clouds, int32_t dim, const fdb_options* opt,
                                       size_t* h_out);
fdb_status fdb_dbscan_batched(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                              int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                              const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* num_clusters,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Out-of-core batch (Section 6 names a batched mode for data and index that do
 * not fit in GPU memory): the clouds stay in host memory and may add up to more
 * than HBM holds. They are clustered in groups of consecutive whole clouds, each
 * group one fdb_dbscan_batched call inside device_budget_bytes: two group slots,
 * so the input copy of one group runs while the previous group is clustered (on
 * a second stream), and results are copied back as groups finish. Every cloud's
 * labels, is_core and K are those fdb_dbscan_batched gives (so those of
 * fdb_dbscan for the cloud alone). Synchronous: returns when all results are in
 * the caller's host buffers.
 *   h_points         host float32, row-major [offsets[num_clouds]][dim]. Pinned
 *                    (page-locked) buffers let copies overlap the clustering;
 *                    pageable ones work, with the copies serialised.
 *   h_offsets        host int64 [num_clouds+1]: offsets[0] = 0, nondecreasing,
 *                    each cloud below 2^30 points (else FDB_ERR_INVALID); the
 *                    total may exceed 2^30.
 *   h_eps, h_min_pts host float32 / int32 [num_clouds], as in fdb_dbscan_batched
 *                    (a cloud with bad values gets K = -1).
 *   device_budget_bytes  device memory the call may allocate: two slots, each
 *                    the largest group's workspace and buffers (at most half the
 *                    budget), freed before returning. A cloud whose batched
 *                    workspace and buffers exceed half the budget gives
 *                    FDB_ERR_NOMEM, before any work.
 *   h_labels         host int32 [total] out; h_is_core host uint8 [total] or NULL;
 *   h_num_clusters   host int32 [num_clouds] out (K, or -1 as in fdb_dbscan_batched).
 * Returns FDB_ERR_INTERNAL if a kernel's consistency check failed in any group;
 * afterwards fdb_last_info reports the bits of all groups together.
 */
fdb_status fdb_dbscan_batched_host(fdb_handle* h, const float* h_points, const int64_t* h_offsets,
                                   int32_t num_clouds, int32_t dim, const float* h_eps, const int32_t* h_min_pts,
                                   const fdb_options* opt, size_t device_budget_bytes, int32_t* h_labels,
                                   uint8_t* h_is_core, int32_t* h_num_clusters);

/* Device-side status of the last call on h: waits for `stream` (the stream that
   call was ordered on, or one ordered after it) and returns its FDB_INFO_* bits in
   *h_info. Returns FDB_ERR_NONFINITE or FDB_ERR_INTERNAL when those bits say the
   labels are undefined, else FDB_OK (also FDB_ERR_HIP, FDB_ERR_INVALID). */
fdb_status fdb_last_status(fdb_handle* h, hipStream_t stream, uint32_t* h_info);

/* fdb_last_status on the stream of the last call, returning FDB_OK whatever the
   bits say (kept for earlier callers). */
fdb_status fdb_last_info(fdb_handle* h, uint32_t* h_info);

/* Wait for the stream of the last fdb_dbscan (or fdb_dbscan_batched) call on h and
   report its sizes, for cost models: h_counts[0] = K (clusters; a batch: summed over
   its clouds), [1] = non-empty grid cells, [2] = dense cells, [3] = BVH primitives
   (dense cells + points outside them; n for FDbscan). Entries 1-2 are 0 for FDbscan.
   The workspace of that call must still be alive. */
fdb_status fdb_last_counts(fdb_handle* h, int64_t* h_counts);

/* Per-stage GPU timing. With timing enabled, fdb_dbscan records a HIP event pair
   around every stage on the call's stream; fdb_stage_times waits for the last
   call and reports up to `max` stages: names (static strings) and milliseconds,
   accumulated over the calls since timing was last enabled or reset, and the
   number of calls in h_calls. */
fdb_status fdb_set_timing(fdb_handle* h, int32_t enable);
fdb_status fdb_stage_times(fdb_handle* h, int32_t max, const char** h_names, double* h_ms, int32_t* h_count,
                           int32_t* h_calls);

/* Test hook (synchronous): count the points of a union-find forest parent[n]
   (device int32, every entry a point index) that break the invariants the fused
   main phase keeps (Section 3.2's union and claim steps, with roots hooked
   smaller-index-first): a core point's parent is a core point with a smaller
   index (or itself), and any other point's parent is itself or a core point;
   an entry outside [0, n) counts too. is_core: device uint8 [n], or NULL when
   every point is core. *h_bad receives the count. */
fdb_status fdb_debug_forest(fdb_handle* h, const int32_t* parent, const uint8_t* is_core, int64_t n,
                            int64_t* h_bad);

/* Test hook (synchronous, allocates; not for production use): build the LBVH over m
   sorted 64-bit keys h_keys (Karras' hierarchy, ties by index; Section 4.1), return
   every internal node's split h_gamma[k] and other range end h_other[k] (k < m-1),
   and walk it from the root with every box accepted, masked at `mask` as in the main
   phase (Section 4.1, Figure 1: subtrees whose leaves are all <= mask are skipped;
   mask = -1 walks everything). h_leaves[0..*h_num_leaves) receives the leaves reached,
   in walk order (h_leaves holds m entries). m <= 2^24. */
fdb_status fdb_debug_lbvh(fdb_handle* h, const uint64_t* h_keys, int32_t m, int32_t mask, int32_t leaf_size,
                          int32_t* h_gamma, int32_t* h_other, int32_t* h_leaves, int32_t* h_num_leaves);

/*
 * Served clustering: a stream of independent jobs (each one cloud with its own
 * eps and minPts, as in fdb_dbscan) on one device. The method itself is the
 * per-cloud clustering of Sections 4.1-4.2; serving many clouds at once is not
 * in the paper. A server owns one worker thread and one device arena of
 * hbm_budget_bytes allocated at creation; jobs never allocate.
 *   FDB_SERVE_BATCHED  continuous batching over two slots, each half the arena
 *                      with its own stream: whenever a slot is free, the worker
 *                      takes the waiting jobs of the oldest job's dim, in arrival
 *                      order, while the batch (its fdb_dbscan_batched workspace
 *                      plus gathered points, labels, flags and per-job arrays)
 *                      fits in the slot and holds at most max_batch jobs, and
 *                      launches them as one batched launch sequence without
 *                      waiting; jobs arriving while it runs go to the other slot,
 *                      so two batches overlap on the device. A job must fit in
 *                      one slot (half the budget).
 *   FDB_SERVE_FIFO     one job at a time with fdb_dbscan, in arrival order (the
 *                      plain server; the arena is its workspace).
 * A job's labels, is_core and K equal what fdb_dbscan gives for it alone
 * (canonical border mode; opt->border = FDB_BORDER_FIRST gives a valid
 * first-claim assignment instead).
 */
typedef struct fdb_server fdb_server;

enum { FDB_SERVE_BATCHED = 0, FDB_SERVE_FIFO = 1 };

typedef struct {
  const float* points; /* device [n][dim] float32; must stay unchanged until the job is done */
  int64_t n;           /* 0 <= n < 2^30; n = 0 completes at submission with K = 0 */
  int32_t dim;         /* 2 or 3 */
  float eps;           /* finite, > 0 */
  int32_t min_pts;     /* >= 1 */
  int32_t* labels;     /* device int32 [n] out (input order; -1 noise, else 0..K-1) */
  uint8_t* is_core;    /* device uint8 [n] out, or NULL */
} fdb_job;

typedef struct {
  int32_t done;         /* 1 once the outputs are final (the device work has completed) */
  int32_t status;       /* fdb_status of the job once done: FDB_OK, FDB_ERR_NONFINITE, ... */
  int32_t num_clusters; /* K once done (-1 when the labels are undefined) */
  int32_t batch_jobs;   /* jobs in the launch that ran it (0 while queued) */
  double queue_us;      /* submission -> start of its batch (-1 while queued) */
  double latency_us;    /* submission -> outputs final (-1 until done) */
} fdb_job_result;

typedef struct {
  int64_t jobs;           /* completed jobs with n > 0 among the tickets counted */
  int64_t points;         /* their points */
  int64_t batches;        /* launches since creation */
  int64_t max_queue;      /* longest queue seen since creation */
  int32_t max_batch_jobs; /* most jobs in one launch since creation */
  double span_s;          /* first submission -> last completion of the counted jobs */
  double busy_s;          /* worker time spent running launches since creation */
  double p50_us, p99_us;  /* latency percentiles (nearest rank) of the counted jobs */
  double mean_us, max_us;
} fdb_serve_stats;

/* Create a server on `device`. max_batch in 1 .. 2^20 (ignored in FIFO mode);
   hbm_budget_bytes >= 1 MiB. FDB_ERR_NOMEM if the arena cannot be allocated. */
fdb_status fdb_server_create(int device, size_t hbm_budget_bytes, int32_t max_batch, int32_t mode,
                             const fdb_options* opt, fdb_server** out);
/* Queue a job (thread-safe, never waits for the device). The job's points must
   be ready on the device (the caller's stream synchronised) before this call.
   FDB_ERR_INVALID for bad arguments, FDB_ERR_NOMEM if the job alone does not fit
   in a slot (batched mode: half the budget; FIFO: the budget). *h_ticket identifies
   the job (0, 1, 2, ... in submission order). */
fdb_status fdb_server_submit(fdb_server* s, const fdb_job* job, int64_t* h_ticket);
/* State of a job without waiting, or waiting until it is done (h_out may be NULL). */
fdb_status fdb_server_poll(fdb_server* s, int64_t ticket, fdb_job_result* h_out);
fdb_status fdb_server_wait(fdb_server* s, int64_t ticket, fdb_job_result* h_out);
/* Wait until every job submitted so far is done. */
fdb_status fdb_server_drain(fdb_server* s);
/* Latency and throughput over the jobs with ticket >= first_ticket (e.g. to leave
   out a warm-up period). */
fdb_status fdb_server_stats(fdb_server* s, int64_t first_ticket, fdb_serve_stats* h_out);
/* Run every queued job, stop the worker and free the server's memory. */
void fdb_server_destroy(fdb_server* s);

/*
 * Autotuner for the launch shape (leaf_size, block_size, tile of fdb_options;
 * none of them changes any label). Times the call on the caller's own input:
 * first the default shape, then coordinate descent over leaf_size in {4, 8, 16,
 * 32}, block_size in {64, 128, 256} and tile in {32, 64}, each shape timed as the
 * median of `reps` (1..100) runs after one warm-up, with HIP events on `stream`.
 * The fastest shape is kept in the handle for the call's class - algorithm
 * (the automatic choice counts as DenseBox), dim, floor(log2 n), minPts <= 2 or
 * not, and for fdb_tune_batched a batch flag with n = n_total - so later calls of
 * that class with 0 in those fields take it. If the environment variable
 * FDB_TUNE_CACHE names a file, the result is appended to it as one text line,
 * and fdb_create reads the file back (later lines win). Arguments are those of
 * fdb_dbscan / fdb_dbscan_batched (the outputs receive the labels of the last
 * run); *h_best receives the chosen options, h_ms[0] their time and h_ms[1] the
 * default shape's time, in ms. Synchronous. FDB_ERR_INVALID also for n < 1.
 */
fdb_status fdb_tune(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                    const fdb_options* opt, int32_t reps, int32_t* labels, uint8_t* is_core, void* workspace,
                    size_t workspace_bytes, hipStream_t stream, fdb_options* h_best, double* h_ms);
fdb_status fdb_tune_batched(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                            int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                            const fdb_options* opt, int32_t reps, int32_t* labels, uint8_t* is_core,
                            int32_t* num_clusters, void* workspace, size_t workspace_bytes, hipStream_t stream,
                            fdb_options* h_best, double* h_ms);
/* The options a call would run with: opt (NULL = all-zero) with the launch-shape
   fields left at 0 filled from the handle's tuned table (num_clouds = 0 for
   fdb_dbscan, else the batch's cloud count), then from the built-in defaults. */
fdb_status fdb_tuned_options(fdb_handle* h, int64_t n, int32_t dim, int32_t min_pts, int32_t num_clouds,
                             const fdb_options* opt, fdb_options* h_out);

/* Static description of a status code. */
const char* fdb_status_string(fdb_status s);

#ifdef __cplusplus
}
#endif

#endif /* FDBSCAN_H */
