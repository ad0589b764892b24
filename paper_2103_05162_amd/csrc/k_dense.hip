// FDbscan-DenseBox preprocessing (Section 4.2). Points arrive sorted by grid-cell
// key (cells of side eps/sqrt(d), keyed along a Morton curve), so each cell is a
// contiguous run. A cell is dense when it holds at least minPts points; then all
// its points are core and share one cluster. The BVH is built over a mix of
// dense-cell boxes and the points outside dense cells, in key order, so the one
// sort serves both the grid and the tree.
//
// Exactness guard (the paper asks for one, Section 4.2): a cell counts as dense
// only if the neighbour test holds across its tight bounding box's diagonal,
// evaluated with the same fp32 operations. Rounded subtraction is monotone, so
// then every pair of points in the cell passes the test, whatever rounding the
// cell index computation suffered.
#include <algorithm>

#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

constexpr int kBlock = 256;

// Sorted keys as 32- or 64-bit words: the width is fixed by the caller (key64) or,
// for a DenseBox grid sized on the device, read from the plan's flag (d_key64).
struct KeyIn {
  const void* p;
  const int* d_key64;
  int key64;
  __device__ __forceinline__ bool wide() const { return d_key64 ? *d_key64 != 0 : key64 != 0; }
};
__device__ __forceinline__ uint64_t key_at(const KeyIn& k, bool wide, int64_t i) {
  return wide ? static_cast<const uint64_t*>(k.p)[i] : static_cast<const uint32_t*>(k.p)[i];
}

// Per-cloud parameters of a batch (null cl_minpts: one cloud with the scalars).
struct CloudParams {
  const uint64_t* keys;  // sorted point keys; cloud = key >> shift
  int shift;
  const int* minpts;
  const float* eps2;
};

__device__ __forceinline__ int cell_minpts(const CloudParams& cp, int head, int min_pts) {
  return cp.minpts ? cp.minpts[cp.keys[head] >> cp.shift] : min_pts;
}
__device__ __forceinline__ float cell_eps2(const CloudParams& cp, int head, float eps2) {
  return cp.eps2 ? cp.eps2[cp.keys[head] >> cp.shift] : eps2;
}

constexpr int kSmallCell = 64;

__device__ __forceinline__ bool is_head(const KeyIn& k, bool wide, int64_t i) {
  return i == 0 || key_at(k, wide, i) != key_at(k, wide, i - 1);
}

// The stage runs as two scans over tiles of kScanTile sorted points (256 threads x
// kScanItems): first over cell heads (a point whose key differs from the one
// before it), giving every point its cell and every cell its start; then, once the
// cells are decided, over primitive openings (a point outside dense cells, or a
// dense cell's first point) and dense-cell openings, giving every primitive its
// index and every dense cell its place in the dense list. Each scan is a reduce
// kernel (one count per tile), a scan of the tile counts, and an apply kernel that
// rescans its tile in LDS and writes the results.

// Tile position p lives at LDS word p + p/16, so a thread's blocked run of 16
// positions falls on distinct banks while global memory is read striped.
__device__ __forceinline__ int tile_lds(int p) { return p + (p >> 4); }

__device__ __forceinline__ int wave_incl(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ int tile_reduce(int x, int* s_w) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  int t = 0;
  for (int j = 0; j < kBlock / 64; ++j) t += s_w[j];
  return t;
}

// Exclusive scan of the tile held in s_v (tile_lds layout), in place; values are
// sums of packed counters, each field below 2^16 over a tile.
__device__ __forceinline__ void tile_exclusive_scan(int* s_v, int* s_w) {
  const int tid = threadIdx.x;
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = s_v[tid * (kScanItems + 1) + k];
    sum += v[k];
  }
  const int inc = wave_incl(sum);
  const int w = tid >> 6;
  if ((tid & 63) == 63) s_w[w] = inc;
  __syncthreads();
  int run = inc - sum;
  for (int j = 0; j < w; ++j) run += s_w[j];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    s_v[tid * (kScanItems + 1) + k] = run;
    run += v[k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_heads_reduce(KeyIn keys, int64_t n, int* __restrict__ bsums) {
  __shared__ int s_w[kBlock / 64];
  const bool wide = keys.wide();
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  int x = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n && is_head(keys, wide, i)) ++x;
  }
  const int t = tile_reduce(x, s_w);
  if (threadIdx.x == 0) bsums[blockIdx.x] = t;
}

// cell_id[i] for every point; cell_start[c] for every cell and cell_start[#cells] = n.
__global__ __launch_bounds__(kBlock) void k_heads_apply(KeyIn keys, int64_t n, const int* __restrict__ bsums,
                                                        int* __restrict__ cell_id, int* __restrict__ cell_start) {
  static_assert(kScanItems == 16, "the LDS layout assumes 16 items per thread");
  __shared__ int s_v[kScanTile + kScanTile / 16];
  __shared__ int s_w[kBlock / 64];
  const bool wide = keys.wide();
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  const int tid = threadIdx.x;
  uint32_t hmask = 0;  // bit k: striped item k is a head
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i = base + p;
    const bool h = i < n && is_head(keys, wide, i);
    hmask |= h ? 1u << k : 0u;
    s_v[tile_lds(p)] = h ? 1 : 0;
  }
  __syncthreads();
  tile_exclusive_scan(s_v, s_w);
  const int carry = bsums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i = base + p;
    if (i < n) {
      const bool h = (hmask >> k) & 1u;
      const int c = carry + s_v[tile_lds(p)] + (h ? 1 : 0) - 1;
      cell_id[i] = c;
      if (h) cell_start[c] = static_cast<int>(i);
      if (i == n - 1) cell_start[c + 1] = static_cast<int>(n);
    }
  }
}

// Per cell: not a candidate (fewer than minPts points) -> not dense; a candidate
// of at most kSmallCell points -> tight box over eight lanes, then the guard;
// a larger candidate -> listed for the wavefront-per-cell kernel. Eight cells
// per wavefront, so the many one-point cells cost little.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cells_small(const float* __restrict__ xs, int64_t n,
                                                        const int* __restrict__ cell_start,
                                                        const int* __restrict__ d_cells, int min_pts, float eps2_all,
                                                        CloudParams cp, uint8_t* __restrict__ dense,
                                                        float4* __restrict__ cell_lo, float4* __restrict__ cell_hi,
                                                        int* __restrict__ big, int* __restrict__ num_big) {
  constexpr int G = 8;
  const int ncells = *d_cells;
  const int sub = threadIdx.x & (G - 1);
  for (int64_t c0 = blockIdx.x * int64_t(kBlock / G); c0 < ncells; c0 += int64_t(gridDim.x) * (kBlock / G)) {
    const int64_t c = c0 + threadIdx.x / G;
    const bool valid = c < ncells;
    int s = 0, e = 0;
    bool cand = false;
    if (valid) {
      s = cell_start[c];
      e = cell_start[c + 1];
      cand = e - s >= cell_minpts(cp, s, min_pts);
    }
    const bool large = cand && e - s > kSmallCell;
    const bool small = cand && !large;
    if (small) {  // the group's eight lanes share c, so they are active together
      float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int j0 = s + sub; j0 < e; j0 += 4 * G) {
        float v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * G;
#pragma unroll
          for (int k = 0; k < D; ++k) v[u][k] = j < e ? xs[k * n + j] : NAN;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < D; ++k) {
            lo[k] = fminf(lo[k], v[u][k]);  // fminf/fmaxf ignore the NaN fill
            hi[k] = fmaxf(hi[k], v[u][k]);
          }
      }
#pragma unroll
      for (int k = 0; k < D; ++k)
        for (int off = G / 2; off > 0; off >>= 1) {
          lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
          hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
      if (sub == 0) {
        if (D == 2) lo[2] = hi[2] = 0.0f;
        const float eps2 = cell_eps2(cp, s, eps2_all);
        dense[c] = dist2v<D>(hi[0], hi[1], hi[2], lo[0], lo[1], lo[2]) <= eps2 ? 1 : 0;
        cell_lo[c] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        cell_hi[c] = make_float4(hi[0], hi[1], hi[2], 0.0f);
      }
    } else if (valid && sub == 0) {
      dense[c] = 0;  // a large candidate is decided by k_cell_boxes
    }
    // list the large candidates: one atomic per wavefront
    const bool push = large && sub == 0;
    const uint64_t bm = ballot(push);
    if (bm) {
      const int leader = __ffsll(static_cast<unsigned long long>(bm)) - 1;
      int at = 0;
      if (lane_id() == leader) at = atomicAdd(num_big, __popcll(bm));
      at = __shfl(at, leader);
      if (push) big[at + __popcll(bm & lanemask_lt())] = static_cast<int>(c);
    }
  }
}

// Opening flags of point i: bit 0 a primitive (outside dense cells, or a dense
// cell's first point), bit 16 a dense cell (its first point).
__device__ __forceinline__ int open_flags(const int* __restrict__ cell_id, const int* __restrict__ cell_start,
                                          const uint8_t* __restrict__ dense, int64_t i, int* c_out, bool* d_out) {
  const int c = cell_id[i];
  const bool d = dense[c] != 0;
  const bool first = cell_start[c] == i;
  *c_out = c;
  *d_out = d;
  return (!d || first ? 1 : 0) | (d && first ? 1 << 16 : 0);
}

__global__ __launch_bounds__(kBlock) void k_prims_reduce(const int* __restrict__ cell_id,
                                                         const int* __restrict__ cell_start,
                                                         const uint8_t* __restrict__ dense, int64_t n,
                                                         int* __restrict__ bsums_p, int* __restrict__ bsums_d) {
  __shared__ int s_w[kBlock / 64];
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  int x = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n) {
      int c;
      bool d;
      x += open_flags(cell_id, cell_start, dense, i, &c, &d);
    }
  }
  const int t = tile_reduce(x, s_w);
  if (threadIdx.x == 0) {
    bsums_p[blockIdx.x] = t & 0xffff;
    bsums_d[blockIdx.x] = t >> 16;
  }
}

// Primitive records in key order (DenseBox leaf records: a point's coordinates
// and index, or a dense cell's low corner and -2 - its first point, beside its
// high corner), the dense list (dense cells' primitive indices, in key order),
// and the union-find start: a dense cell's points hang under its first point and
// are core by construction; every other point starts alone.
template <int D>
__global__ __launch_bounds__(kBlock) void k_prims_apply(KeyIn keys, const float* __restrict__ xs, int64_t n,
                                                        const int* __restrict__ cell_id,
                                                        const int* __restrict__ cell_start,
                                                        const uint8_t* __restrict__ dense,
                                                        const float4* __restrict__ cell_lo,
                                                        const float4* __restrict__ cell_hi,
                                                        const int* __restrict__ bsums_p, const int* __restrict__ bsums_d,
                                                        int* __restrict__ prim_start, int* __restrict__ prim_cnt,
                                                        float4* __restrict__ prim_lo, float4* __restrict__ prim_hi,
                                                        uint64_t* __restrict__ prim_key, int* __restrict__ dense_list,
                                                        int* __restrict__ labels, uint8_t* __restrict__ core,
                                                        int* __restrict__ pidx, int* __restrict__ ends,
                                                        int* __restrict__ minorig) {
  __shared__ int s_v[kScanTile + kScanTile / 16];
  __shared__ int s_w[kBlock / 64];
  const bool wide = keys.wide();
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  const int tid = threadIdx.x;
  int cl[kScanItems];
  uint32_t dmask = 0;  // bit k: striped item k lies in a dense cell
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i = base + p;
    int f = 0;
    cl[k] = 0;
    if (i < n) {
      bool d;
      f = open_flags(cell_id, cell_start, dense, i, &cl[k], &d);
      dmask |= d ? 1u << k : 0u;
    }
    s_v[tile_lds(p)] = f;
  }
  __syncthreads();
  // the flags are needed again after the scan: keep them per item
  int fl[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) fl[k] = s_v[tile_lds(k * kBlock + tid)];
  __syncthreads();
  tile_exclusive_scan(s_v, s_w);
  const int carry_p = bsums_p[blockIdx.x], carry_d = bsums_d[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i64 = base + p;
    if (i64 >= n) continue;
    const int i = static_cast<int>(i64);
    const int ex = s_v[tile_lds(p)];
    const int pi = carry_p + (ex & 0xffff);
    if (pidx) pidx[i] = pi;  // primitives opened before point i (a batch finds its clouds' subtrees with it)
    // starting values the hierarchy build and the finalisation expect, written here
    // instead of in fills of their own
    if (minorig) minorig[i] = 0x7fffffff;
    if (ends && (fl[k] & 1)) ends[pi] = -1;
    const bool d = (dmask >> k) & 1u;
    if (d) {
      const int c = cl[k];
      const int st = cell_start[c];
      labels[i] = st;
      core[i] = 1;
      if (fl[k] >> 16) {  // the cell's first point opens its primitive
        const float4 lo = cell_lo[c], hi = cell_hi[c];
        const int np = cell_start[c + 1] - st;
        prim_start[pi] = st;
        prim_cnt[pi] = -np;
        prim_lo[pi] = make_float4(lo.x, lo.y, lo.z, __int_as_float(-2 - st));
        prim_hi[pi] = make_float4(hi.x, hi.y, hi.z, __int_as_float(np));  // w: the cell's point count
        prim_key[pi] = key_at(keys, wide, i);
        dense_list[carry_d + (ex >> 16)] = pi;
      }
    } else {
      labels[i] = i;
      core[i] = 0;
      prim_start[pi] = i;
      prim_cnt[pi] = 1;
      prim_lo[pi] = make_float4(xs[i], xs[n + i], D == 3 ? xs[2 * n + i] : 0.0f, __int_as_float(i));
      prim_key[pi] = key_at(keys, wide, i);
    }
  }
}

// Tight box of each listed cell of more than kSmallCell points, a wavefront per
// cell (G = 64 lanes), then the guard.

template <int D, int G>
__global__ __launch_bounds__(kBlock) void k_cell_boxes(const float* __restrict__ xs, int64_t n,
                                                       const int* __restrict__ cell_start, const int* __restrict__ cand,
                                                       const int* __restrict__ num_cand, float eps2_all,
                                                       CloudParams cp, uint8_t* __restrict__ dense,
                                                       float4* __restrict__ cell_lo, float4* __restrict__ cell_hi) {
  const int sub = threadIdx.x & (G - 1);
  const int grp = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int ngrp = (gridDim.x * kBlock) / G;
  const int ncand = *num_cand;
  for (int w = grp; w < ncand; w += ngrp) {
    const int c = cand[w];
    const int s = cell_start[c], e = cell_start[c + 1];
    if ((e - s > kSmallCell) != (G == 64)) continue;  // the other launch takes it
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    // four G-point chunks per trip: their loads are in flight together
    for (int j0 = s + sub; j0 < e; j0 += 4 * G) {
      float v[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u * G;
#pragma unroll
        for (int k = 0; k < D; ++k) v[u][k] = j < e ? xs[k * n + j] : NAN;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          lo[k] = fminf(lo[k], v[u][k]);  // fminf/fmaxf ignore the NaN fill
          hi[k] = fmaxf(hi[k], v[u][k]);
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
      for (int off = G / 2; off > 0; off >>= 1) {  // within the group (its lanes run together)
        lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
        hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
      }
    if (sub == 0) {
      if (D == 2) lo[2] = hi[2] = 0.0f;
      const float eps2 = cell_eps2(cp, s, eps2_all);
      bool ok = dist2v<D>(hi[0], hi[1], hi[2], lo[0], lo[1], lo[2]) <= eps2;
      dense[c] = ok ? 1 : 0;
      cell_lo[c] = make_float4(lo[0], lo[1], lo[2], 0.0f);
      cell_hi[c] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    }
  }
}

void cells_t(const KeyIn& keys, int64_t n, int dim, const float* xs, float eps2, int min_pts, int* cell_id,
             int* cell_start, int* cand, uint8_t* dense, float4* cell_lo, float4* cell_hi, int* pflag,
             int* prim_start, int* prim_cnt, float4* prim_lo, float4* prim_hi, uint64_t* prim_key, int* dense_list,
             int* labels, uint8_t* core, int* misc, int* bsums, int64_t scan_blocks, const CloudParams& cp,
             hipStream_t s, int* ends, int* minorig) {
  (void)scan_blocks;
  int* d_cells = misc + kMiscNumCells;
  int* d_big = misc + kMiscNumCand;  // candidate cells of more than kSmallCell points
  int* d_prims = misc + kMiscNumPrims;
  int* d_dense = misc + kMiscNumDense;
  const int64_t tiles = ceil_div(n, kScanTile);
  const dim3 gt(static_cast<unsigned>(tiles));
  hipLaunchKernelGGL(k_heads_reduce, gt, dim3(kBlock), 0, s, keys, n, bsums);
  scan_block_sums(bsums, tiles, d_cells, s);
  hipLaunchKernelGGL(k_heads_apply, gt, dim3(kBlock), 0, s, keys, n, bsums, cell_id, cell_start);
  // d_big (a misc slot) is zero: the caller cleared misc before this stage
  int* big = cand;
  const int gs = static_cast<int>(std::min<int64_t>(std::max<int64_t>(ceil_div(n, kBlock / 8), 1), 8192));
  const int gb = 2048;  // 8192 wavefronts, grid-stride over the listed cells
  if (dim == 3) {
    hipLaunchKernelGGL(k_cells_small<3>, dim3(gs), dim3(kBlock), 0, s, xs, n, cell_start, d_cells, min_pts, eps2, cp,
                       dense, cell_lo, cell_hi, big, d_big);
    hipLaunchKernelGGL((k_cell_boxes<3, 64>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, big, d_big, eps2, cp,
                       dense, cell_lo, cell_hi);
  } else {
    hipLaunchKernelGGL(k_cells_small<2>, dim3(gs), dim3(kBlock), 0, s, xs, n, cell_start, d_cells, min_pts, eps2, cp,
                       dense, cell_lo, cell_hi, big, d_big);
    hipLaunchKernelGGL((k_cell_boxes<2, 64>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, big, d_big, eps2, cp,
                       dense, cell_lo, cell_hi);
  }
  int* bsums_d = pflag;  // the dense-cell counts of each tile
  // a batch reads every point's primitive index afterwards (in cand, which the
  // large-cell list no longer needs by then)
  int* pidx = cp.minpts ? cand : nullptr;
  hipLaunchKernelGGL(k_prims_reduce, gt, dim3(kBlock), 0, s, cell_id, cell_start, dense, n, bsums, bsums_d);
  scan_block_sums(bsums, tiles, d_prims, s, bsums_d, d_dense);
  if (dim == 3)
    hipLaunchKernelGGL(k_prims_apply<3>, gt, dim3(kBlock), 0, s, keys, xs, n, cell_id, cell_start, dense, cell_lo,
                       cell_hi, bsums, bsums_d, prim_start, prim_cnt, prim_lo, prim_hi, prim_key, dense_list, labels,
                       core, pidx, ends, minorig);
  else
    hipLaunchKernelGGL(k_prims_apply<2>, gt, dim3(kBlock), 0, s, keys, xs, n, cell_id, cell_start, dense, cell_lo,
                       cell_hi, bsums, bsums_d, prim_start, prim_cnt, prim_lo, prim_hi, prim_key, dense_list, labels,
                       core, pidx, ends, minorig);
}

}  // namespace

void densebox_cells(const void* sorted_keys, bool key64, const int* d_key64, int64_t n, int dim, const float* xs,
                    float eps2, int min_pts, int* cell_id, int* cell_start, int* cand, uint8_t* cell_dense,
                    float4* cell_lo, float4* cell_hi, int* pflag, int* prim_start, int* prim_cnt, float4* prim_lo,
                    float4* prim_hi, uint64_t* prim_key, int* dense_list, int* labels, uint8_t* core, int* misc,
                    int* bsums, int64_t scan_blocks, hipStream_t s, int key_shift, const int* cl_minpts,
                    const float* cl_eps2, int* ends, int* minorig) {
  // per-cloud parameters come with batches, whose keys are always 64-bit
  CloudParams cp{static_cast<const uint64_t*>(sorted_keys), key_shift, cl_minpts, cl_eps2};
  const KeyIn keys{sorted_keys, d_key64, key64 ? 1 : 0};
  cells_t(keys, n, dim, xs, eps2, min_pts, cell_id, cell_start, cand, cell_dense, cell_lo, cell_hi, pflag, prim_start,
          prim_cnt, prim_lo, prim_hi, prim_key, dense_list, labels, core, misc, bsums, scan_blocks, cp, s, ends,
          minorig);
}

}  // namespace fdb
