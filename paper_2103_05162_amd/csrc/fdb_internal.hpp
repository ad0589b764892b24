// Host-side internals of libfdbscan: the workspace plan, the device views the
// kernels receive, and the launch helpers each kernel file exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct fdb_handle;

namespace fdb {

// Keys per thread in a radix pass, by key width (measured: 64-bit keys fit two
// 6144-key tiles per CU in LDS; 32-bit keys do best at 5120). The workspace
// sizes the look-back status for the smaller tile.
template <typename K>
constexpr int sort_items() { return sizeof(K) == 8 ? 24 : 22; }
constexpr int kSortTileMin = 256 * 20;  // smallest keys-per-workgroup tile
constexpr int kScanItems = 16;                 // items per thread in the device scan
constexpr int kScanTile = 256 * kScanItems;
constexpr int64_t kMaxPoints = (int64_t(1) << 30) - 1;
constexpr int kRecNb = 8;  // neighbouring primitives recorded per non-core point

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Byte offsets of every buffer inside the caller's (or the handle's) workspace.
// Sizes depend on (n, dim, algo) only, never on eps or minPts: the footprint is
// linear in n (Section 3.2).
struct Plan {
  int64_t n = 0;
  int dim = 3;
  int algo = 0;
  size_t bytes = 0;
  // common
  size_t bounds, misc, gplan, keys0, keys1, vals0, vals1, hist, digoff, tilectr, status;
  size_t xs;                       // dim * n floats, sorted SoA
  size_t node_a, node_b, rope, leaf_rope, ends, other, gamma, cut;
  size_t labels, core, lone, qborder, brec_i, brec_nb;
  int64_t brec_cap = 0;
  size_t minorig, lflag, rank, bsums, cid, border;
  // DenseBox
  size_t cell_id, cell_start, cand, cell_dense, cell_lo, cell_hi, pflag, prim_start, prim_cnt,
      prim_lo, prim_hi, prim_key, dense_list;
  // batches
  int num_clouds = 0;
  size_t cl_lo, cl_scale, cl_eps2, cl_minpts, cl_root, cl_end, cl_flags, cl_ord;
  int64_t sort_tiles = 0, scan_blocks = 0;
  int64_t map_bytes = 0;  // DenseBox: bytes from cell_lo to the end of cell_hi (free after the primitives)
};

Plan make_plan(int64_t n, int dim, int algo, int num_clouds = 0);

// Small device-side scalars kept in the workspace's misc block.
enum MiscSlot : int {
  kMiscNumClusters = 0,  // K after the scan
  kMiscNumCells = 1,     // DenseBox: number of non-empty cells
  kMiscNumCand = 2,      // DenseBox: cells with >= minPts points
  kMiscNumPrims = 3,     // DenseBox: m = dense cells + points outside them
  kMiscNumDense = 4,     // DenseBox: dense cells
  kMiscBorderQ = 5,      // entries of the border query list (filled by the core pass)
  kMiscBorderRec = 6,    // border neighbour records asked for by the core pass
  kMiscCut = 7,          // entries of the hierarchy's cut (TreeView::cut)
  kMiscCoreQ = 8,        // DenseBox: point primitives left for the core pass by the isolated-point test,
                         // one count per XCD segment (slots 8 .. 15)
  kMiscCount = 16
};

// DenseBox grid of one cloud (Section 4.2: cells of side eps/sqrt(d)), sized on
// the device from the scene bounds by k_grid_plan, so no value goes back to the
// host mid-call. The key, sort, dense-cell and isolated-point kernels read it.
// When the eps/sqrt(d) grid needs more cells per axis than a 64-bit key holds
// (21 bits per axis in 3D, 31 in 2D), the cells are widened to fit (coarse = 1,
// FDB_INFO_DENSEBOX_FALLBACK): density is still decided by the exact guard, so
// labels stay exact; only fewer cells come out dense.
struct GridPlan {
  float inv_h[4];      // 1 / cell side, per axis
  uint32_t ncell[4];   // cells per axis (>= 1)
  int32_t bits;        // key bits per axis
  int32_t key64;       // 1: d * bits > 32, keys are stored as 64-bit words, else 32-bit
  int32_t passes;      // 8-bit radix passes over the d * bits key bits
  int32_t start;       // key buffer (0/1) the key kernel fills: the sort then ends in buffer 1
  int32_t lone_on;     // the isolated-point test runs (32-bit keys, its map and table fit their buffers)
  int32_t coarse;      // cells widened to fit 64-bit keys
  int64_t lone_words;  // the test's 64-bit occupancy words, one per brick of 64 grid cells
  float reach;         // eps / side plus rounding slack, in cell units (< 2)
};

// Node records are interleaved: node k's two halves sit at node_a[kNodeStride * k]
// and node_b[kNodeStride * k] with node_b = node_a + 1, so a node is 32
// contiguous bytes (one cache line) rather than two lines in two arrays.
constexpr int kNodeStride = 2;

// Device view of an LBVH over m primitives. Internal node k: node_a[k] =
// (lo.xyz, other end of its leaf range as int bits), node_b[k] = (hi.xyz, split
// position gamma as int bits); its leaves are [min(k,other), max(k,other)], its
// children cover [first,gamma] and [gamma+1,last]. rope[k] / leaf_rope[l] give
// the next node in depth-first pre-order after that subtree (kEnd at the end).
struct TreeView {
  const float4* node_a;
  const float4* node_b;
  const int* rope;
  const int* leaf_rope;
  int m_cap;       // number of primitives, or an upper bound when d_m is set
  const int* d_m;  // device-side primitive count (DenseBox), or null
  int leaf_size;   // subtrees of at most this many primitives are scanned linearly
  // A cut through the hierarchy (single-cloud trees): the maximal subtrees of at
  // most cut_span(m) primitives, as pairs {lo.xyz, node ref} {hi.xyz, last
  // primitive}, *cut_n of them; a box walk over the whole tree tests these at once
  // instead of descending from the root. Null, or a count above kCutMax: no cut.
  const float4* cut = nullptr;
  const int* cut_n = nullptr;
  // Optional, per cut subtree (FDbscan's main phase): the root that every core point
  // under it had when the summary was taken, kCutNoCore when it holds none, or
  // kCutMixed. A subtree already in a packet's set adds no union and is not walked.
  const int* cut_sum = nullptr;
};

constexpr int kCutMax = 8192;
constexpr int kCutDiv = 256;      // the cut holds about kCutDiv to 2 kCutDiv subtrees
constexpr int kCutDivFine = 4096;  // FDbscan: subtrees of ~m/4096 primitives, smaller than a clump
constexpr int kCutUnroll = 4;     // cut entries a lane loads at once
constexpr int kCutMixed = -1, kCutNoCore = -2;
__host__ __device__ inline int cut_span(int m, int div = kCutDiv) {
  return (m + div - 1) / div > 64 ? (m + div - 1) / div : 64;
}

// ---- launch helpers (stream-ordered, asynchronous) --------------------------
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
// Up to 8 fills of 32-bit words in one launch (a call's counters and flags).
struct FillSeg {
  uint32_t* p;
  uint32_t v;
  int64_t n;
};
struct FillList {
  FillSeg seg[8];
  int count = 0;
  void add(void* p, uint32_t v, int64_t n) {
    if (n > 0) seg[count++] = FillSeg{static_cast<uint32_t*>(p), v, n};
  }
};
void fill_multi(const FillList& L, hipStream_t s);

// k_prep.hip
void launch_bounds(const float* pts, int64_t n, int dim, uint32_t* bounds, uint32_t* info, hipStream_t s);
// The key kernels also count the digits of the `sort_bits`-bit keys for the
// radix sort into hist (ceil(sort_bits / 8) x 256 words, cleared here).
void launch_morton(const float* pts, int64_t n, int dim, const uint32_t* bounds, uint64_t* keys, uint32_t* vals,
                   int sort_bits, uint32_t* hist, hipStream_t s);
// DenseBox of one cloud: k_grid_plan writes *plan from the bounds (after
// launch_bounds; eps is the caller's), then the cell keys go to key buffer
// plan->start as 32- or 64-bit words with the identity permutation, and their
// digits are counted for the sort (hist: 8 x 256 words, cleared here unless the
// caller has, hist_clear = false).
void launch_grid_plan(const uint32_t* bounds, int dim, float eps, int64_t n, int64_t map_bytes, GridPlan* plan,
                      uint32_t* info, hipStream_t s);
void launch_gridkeys(const float* pts, int64_t n, int dim, const uint32_t* bounds, const GridPlan* plan,
                     void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, uint32_t* hist, hipStream_t s,
                     bool hist_clear = true);
void launch_permute(const float* pts, int64_t n, int dim, const uint32_t* perm, float* xs, uint32_t* info,
                    hipStream_t s);

// k_sort.hip: LSD radix sort of (key, index) pairs over the low `bits` bits.
// hist_ready: hist already holds the digit counts of every pass (from the key
// kernel). digoff: 8 * 256 + 8 words (digit offsets, and per pass a flag set when
// every key has the same digit, whose pass then copies instead of sorting).
// Returns which of the two buffers holds the result (0 or 1).
int radix_sort(void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, int64_t n, bool key64, int bits,
               uint32_t* hist, bool hist_ready, uint32_t* digoff, uint32_t* tilectr, uint64_t* status,
               uint32_t* info, hipStream_t s);
// The same with key width and pass count taken from a GridPlan on the device:
// passes for both widths are launched and those the plan does not call for exit
// at once. The keys start in buffer plan->start and end in buffer 1; hist holds
// every pass's digit counts (from the key kernel). The tile counters (8 words)
// and look-back words (planned_status_words(n)) are cleared here unless the
// caller has (clear = false).
void radix_sort_planned(void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, int64_t n, const GridPlan* plan,
                        const uint32_t* hist, uint32_t* digoff, uint32_t* tilectr, uint64_t* status,
                        uint32_t* info, hipStream_t s, bool clear = true);
int64_t planned_status_words(int64_t n);

// k_tree.hip
// prim_lo / prim_hi: DenseBox leaf records (null for FDbscan, whose leaves are
// the sorted points); see TravArgs. ends: m words of scratch; other / gamma:
// each internal node's other range end and split (m - 1 words each). cut / cut_n:
// the cut of TreeView (kCutMax pairs, and a counter the caller zeroed), or null.
void build_lbvh(const void* keys, bool key64, int m, int dim, const float* xs, int64_t n_pts,
                const float4* prim_lo, const float4* prim_hi, float4* node_a, float4* node_b, int* rope,
                int* leaf_rope, int* ends, int* other, int* gamma, const int* d_m, uint32_t* info, hipStream_t s,
                float4* cut = nullptr, int* cut_n = nullptr, bool ends_ready = false, int cut_div = kCutDiv);

// k_dense.hip
// sorted_keys are 64-bit words when key64 (or, with d_key64 set, when *d_key64 on
// the device says so), else 32-bit; prim_key receives each primitive's key as a
// 64-bit word. ends / minorig (optional): set to -1 per primitive and to INT_MAX
// per point, the starting values of build_lbvh's exchange words (pass
// ends_ready) and of launch_finalize's minorig.
void densebox_cells(const void* sorted_keys, bool key64, const int* d_key64, int64_t n, int dim, const float* xs,
                    float eps2, int min_pts, int* cell_id, int* cell_start, int* cand, uint8_t* cell_dense,
                    float4* cell_lo, float4* cell_hi, int* pflag, int* prim_start, int* prim_cnt, float4* prim_lo,
                    float4* prim_hi, uint64_t* prim_key, int* dense_list, int* labels, uint8_t* core, int* misc,
                    int* bsums, int64_t scan_blocks, hipStream_t s, int key_shift = 0,
                    const int* cl_minpts = nullptr, const float* cl_eps2 = nullptr, int* ends = nullptr,
                    int* minorig = nullptr);

// k_trav.hip
struct TravArgs {
  TreeView t;
  const float* xs;  // sorted SoA coordinates: x[n], y[n], z[n]
  int64_t n;
  float eps2;
  float packet_ext_eps2;  // a wavefront walks as one packet if its queries' box extent^2 <= this * eps^2
  int packet_leaf;    // bucket size of packet walks (<= 64: a bucket is loaded one point per lane)
  int min_pts;
  int* labels;
  uint8_t* core;
  uint8_t* lone;  // set by the core pass (or the isolated-point test before it): 1 = not core and no
                  // neighbour but itself (noise); NULL if no core pass
  // Border work left by the core pass for non-core points with some neighbour
  // other than themselves. Up to kRecNb neighbouring primitives of such a point
  // (the point itself, or a dense cell's first point) are recorded, so the
  // border pass needs no walk: record k is point brec_i[k] with neighbours
  // brec_nb[k * kRecNb + t] (-1 = none); *brec_n counts the records asked for,
  // of which the first brec_cap are stored. Points with more neighbouring
  // primitives, or past the capacity, are listed in qborder (DenseBox: their
  // primitive indices) and walk the tree again.
  int* brec_i;
  int* brec_nb;
  int* brec_n;
  int brec_cap;
  int* qborder;
  int* qborder_n;
  const int* cid;
  int* border;
  // DenseBox core pass over lists of point primitives, one per XCD segment
  // (core_list[x * segment + 0 .. core_qn[x]), kNumXcd of them), or over every
  // primitive when core_list is null
  const int* core_list;
  const int* core_qn;
  const int* lone_on;  // device flag: core_list is in use (null = whenever core_list is set)
  // DenseBox primitives (null for FDbscan). Primitive r covers sorted points
  // [prim_start[r], prim_start[r] + |prim_cnt[r]|); prim_cnt > 0: a single
  // point, < 0: a dense cell. prim_lo[r] is the leaf record a walk loads: a
  // point's coordinates with its sorted index as int bits in w (>= 0), or a
  // dense cell's low corner with w = -2 - its first point; prim_hi[r] is a
  // dense cell's high corner.
  const int* prim_start;
  const int* prim_cnt;
  const float4* prim_lo;
  const float4* prim_hi;
  const int* dense_list;  // dense-cell primitive indices
  const int* d_ndense;    // their number (device)
  // batches (null pkeys = one cloud): cloud of sorted point i = pkeys[i] >> key_shift;
  // per cloud: first node and last primitive of its subtree, eps^2, minPts
  const uint64_t* pkeys;
  int key_shift;
  int num_clouds;
  const int* cloud_root;
  const int* cloud_end;
  const float* cloud_eps2;
  const int* cloud_minpts;
  uint32_t* info;  // FDB_INFO_* bits; kernels raise FDB_INFO_INTERNAL on a broken walk
  int block;
};
void launch_core(const TravArgs& a, int dim, bool densebox, hipStream_t s);
// FDbscan, one cloud, before the packet main phase: core pairs among curve
// neighbours joined early, then a summary per cut subtree (kCutMax words at sum;
// a.t.cut must be set) for a.t.cut_sum.
void launch_fdb_local(const TravArgs& a, int dim, bool all_core, hipStream_t s);
void launch_cut_summary(const TravArgs& a, bool all_core, int* sum, hipStream_t s);
// Isolated points before the DenseBox core pass (one cloud, 32-bit grid keys): an
// occupancy map of the grid cells (words: plan->lone_words 64-bit words, one per
// brick of 64 cells, written only for occupied bricks; table: one bit per brick,
// cleared here) settles every point primitive with no occupied cell within reach
// but its own, which it shares with no other primitive: core 0, lone, border -1.
// The others are listed (list, list_n[kNumXcd]) for the core pass. Runs only where
// plan->lone_on; bounds are the scene bounds of launch_bounds.
void launch_lone_filter(const TravArgs& a, int dim, const uint64_t* prim_key, const GridPlan* plan, uint32_t* table,
                        uint64_t* words, const uint32_t* bounds, int* list, int* list_n, hipStream_t s);
void launch_main(const TravArgs& a, int dim, bool densebox, bool all_core, bool first_border, int part,
                 hipStream_t s);
void launch_border(const TravArgs& a, int dim, bool densebox, hipStream_t s);
void launch_debug_walk(const TreeView& t, int m, int mask, int* out_leaves, int* out_count, int cap,
                       uint32_t* info, hipStream_t s);

// k_label.hip
// labels[i] = i; with ends / minorig, also those starting values (see densebox_cells).
void launch_init_labels(int* labels, int64_t n, hipStream_t s, int* ends = nullptr, int* minorig = nullptr);
// With minorig (core flags final): also the smallest input index (perm) of each
// root's core points, in minorig[root] (INT_MAX beforehand, unless minorig_init:
// then filled here first), and the leader words `bits` (ceil(n/32)) cleared.
void launch_finalize(int* labels, int64_t n, uint32_t* info, hipStream_t s, const uint8_t* core = nullptr,
                     const uint32_t* perm = nullptr, int* minorig = nullptr, uint32_t* bits = nullptr,
                     bool minorig_init = true);
void launch_core_from_sets(const int* labels, uint8_t* core, int64_t n, int min_pts, hipStream_t s);
void launch_check_forest(const int* labels, const uint8_t* core, int64_t n, uint32_t* bad, uint32_t* info,
                         hipStream_t s);
// Canonical cluster ids (ids 0..K-1 in increasing order of each cluster's
// smallest core input index). bits: ceil(n/32) leader words followed by as many
// ints of scratch (fits the n-int lflag array); wpre: ceil(n/32) ints.
// minorig_ready: launch_finalize already filled minorig and cleared the leader words.
void canonical_ids(const int* labels, const uint8_t* core, const uint32_t* perm, int64_t n, int* minorig,
                   uint32_t* bits, int* wpre, int* bsums, int64_t scan_blocks, int* cid, int* d_k, hipStream_t s,
                   bool ids = true, bool minorig_ready = false);

// k_batch.hip
void batch_prep(const float* pts, const int64_t* off, int num_clouds, int64_t n, int dim, const float* eps,
                const int32_t* min_pts, int bpd, bool densebox, uint32_t* cl_ord, float4* cl_lo, float4* cl_scale,
                float* cl_eps2, int* cl_minpts, int* cl_flags, uint32_t* info, hipStream_t s);
void batch_keys(const float* pts, const int64_t* off, int num_clouds, int64_t n, int dim, const float4* cl_lo,
                const float4* cl_scale, int bpd, int shift, uint64_t* keys, uint32_t* vals, int sort_bits,
                uint32_t* hist, hipStream_t s);
void batch_roots(const int64_t* off, int num_clouds, int64_t n, const int* pidx, const int* d_m, const int* other,
                 int* root, int* end, uint32_t* info, hipStream_t s);
void batch_cluster_ids(const int* labels, const uint8_t* core, const int* minorig, const uint32_t* bits,
                       const int* wpre, const uint64_t* pkeys, int shift, const int64_t* off, int num_clouds,
                       int64_t n, const int* total, const int* cl_flags, int* cid, int32_t* num_clusters,
                       hipStream_t s);
void launch_scatter(const int* labels, const uint8_t* core, const uint32_t* perm, const int* cid,
                    const int* border, bool first_border, bool have_border, int64_t n, int32_t* out_labels,
                    uint8_t* out_core, uint32_t* info, hipStream_t s);
// The device word of FDB_INFO_* bits that a handle's calls raise (for copies
// ordered on a stream; the server reads its batches' bits this way).
const uint32_t* handle_info(const fdb_handle* h);

// Exclusive scan of blocks int32 counts in place (one workgroup); the total goes to *d_total.
// With bsums2, a second array of as many counts is scanned by a second workgroup of
// the same launch (its total to *d_total2).
void scan_block_sums(int* bsums, int64_t blocks, int* d_total, hipStream_t s, int* bsums2 = nullptr,
                     int* d_total2 = nullptr);
void device_scan(const int* in, int* out, int64_t n, const int* d_n, int* bsums, int64_t blocks, int* d_total,
                 hipStream_t s);

// k_serve.hip: one job of a served batch - its own buffers and its place in the
// batch (first point off; first workgroup gblk of the gather and sblk of the
// scatter, each workgroup moving kSegVec * 256 elements).
constexpr int kSegVec = 4;
struct JobSeg {
  const float* points;
  int32_t* labels;
  uint8_t* core;
  int64_t n;
  int64_t off;
  int32_t gblk, sblk;
};
int64_t seg_blocks(int64_t elems);
void launch_gather(const JobSeg* seg, int num, int64_t total_blocks, int dim, float* dst, hipStream_t s);
void launch_scatter_jobs(const JobSeg* seg, int num, int64_t total_blocks, const int32_t* labels,
                         const uint8_t* core, hipStream_t s);

}  // namespace fdb
