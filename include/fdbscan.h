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
 *   - a handle is used by one host thread at a time.
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
  FDB_ERR_INTERNAL = 5   /* a kernel's own consistency check failed (reported when the call waits) */
} fdb_status;

typedef enum {
  FDB_ALGO_FDBSCAN = 0,  /* LBVH over all points (Section 4.1) */
  FDB_ALGO_DENSEBOX = 1  /* LBVH over dense eps/sqrt(d) grid cells + other points (Section 4.2) */
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
  FDB_BORDER_FIRST = 1
} fdb_border;

typedef struct {
  int32_t algo;       /* fdb_algo */
  int32_t border;     /* fdb_border */
  int32_t leaf_size;  /* traversal: subtrees of <= leaf_size primitives are scanned linearly; 0 = default */
  int32_t block_size; /* threads per workgroup of the traversal kernels (64..1024, multiple of 64); 0 = default */
  uint32_t flags;     /* reserved, must be 0 */
} fdb_options;        /* all-zero = FDbscan, canonical labels, defaults */

/* Information bits, read with fdb_last_info(). */
enum {
  FDB_INFO_DENSEBOX_FALLBACK = 1u, /* DenseBox asked for, but the grid could not be indexed in 64-bit
                                      keys (eps tiny against the extent): FDbscan ran instead. */
  FDB_INFO_NONFINITE = 2u,         /* a NaN or infinite coordinate was seen; labels are undefined */
  FDB_INFO_INTERNAL = 4u           /* a kernel stopped a walk that broke its own bounds; labels undefined */
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
 * DenseBox reads the scene bounds back to the host once (it sizes the grid from
 * them), so with algo = FDB_ALGO_DENSEBOX the call waits for the stream midway.
 */
fdb_status fdb_dbscan(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                      const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                      void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Wait for the stream of the last fdb_dbscan call on h and return its FDB_INFO_* bits. */
fdb_status fdb_last_info(fdb_handle* h, uint32_t* h_info);

/* Wait for the stream of the last fdb_dbscan call on h and report its sizes, for
   cost models: h_counts[0] = K (clusters), [1] = non-empty grid cells, [2] = dense
   cells, [3] = BVH primitives (dense cells + points outside them; n for FDbscan).
   Entries 1-2 are 0 for FDbscan. The workspace of that call must still be alive. */
fdb_status fdb_last_counts(fdb_handle* h, int64_t* h_counts);

/* Per-stage GPU timing. With timing enabled, fdb_dbscan records a HIP event pair
   around every stage on the call's stream; fdb_stage_times waits for the last
   call and reports up to `max` stages: names (static strings) and milliseconds,
   accumulated over the calls since timing was last enabled or reset, and the
   number of calls in h_calls. */
fdb_status fdb_set_timing(fdb_handle* h, int32_t enable);
fdb_status fdb_stage_times(fdb_handle* h, int32_t max, const char** h_names, double* h_ms, int32_t* h_count,
                           int32_t* h_calls);

/* Test hook (synchronous, allocates; not for production use): build the LBVH over m
   sorted 64-bit keys h_keys (Karras' hierarchy, ties by index; Section 4.1), return
   every internal node's split h_gamma[k] and other range end h_other[k] (k < m-1),
   and walk it from the root with every box accepted, masked at `mask` as in the main
   phase (Section 4.1, Figure 1: subtrees whose leaves are all <= mask are skipped;
   mask = -1 walks everything). h_leaves[0..*h_num_leaves) receives the leaves reached,
   in walk order (h_leaves holds m entries). m <= 2^24. */
fdb_status fdb_debug_lbvh(fdb_handle* h, const uint64_t* h_keys, int32_t m, int32_t mask, int32_t leaf_size,
                          int32_t* h_gamma, int32_t* h_other, int32_t* h_leaves, int32_t* h_num_leaves);

/* Static description of a status code. */
const char* fdb_status_string(fdb_status s);

#ifdef __cplusplus
}
#endif

#endif /* FDBSCAN_H */
