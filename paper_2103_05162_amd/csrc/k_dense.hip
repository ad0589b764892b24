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

__global__ __launch_bounds__(kBlock) void k_cell_heads(KeyIn keys, int64_t n, int* __restrict__ head) {
  const bool wide = keys.wide();
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    head[i] = (i == 0 || key_at(keys, wide, i) != key_at(keys, wide, i - 1)) ? 1 : 0;
}

// cell_id[i] = (number of heads at or before i) - 1; heads record their start.
__global__ __launch_bounds__(kBlock) void k_cell_start(const int* __restrict__ head, int64_t n,
                                                       int* __restrict__ cell_id, int* __restrict__ cell_start,
                                                       const int* __restrict__ num_cells) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    int h = head[i];
    int c = cell_id[i] + h - 1;  // cell_id holds the exclusive scan of head on entry
    cell_id[i] = c;
    if (h) cell_start[c] = static_cast<int>(i);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cell_start[*num_cells] = static_cast<int>(n);
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

// Append value to list (counter *n) on every thread where pred holds: one
// atomic per workgroup, threads in order within it (lists stay roughly in key
// order). Every thread of the workgroup must call it; s_w holds 17 ints. Many
// workgroups appending to one counter serialise on it, so the kernels using
// this run 1024-thread workgroups.
constexpr int kPushBlock = 1024;
__device__ __forceinline__ void block_push(int* list, int* n, bool pred, int value, int* s_w) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t b = ballot(pred);
  if (lane_id() == 0) s_w[w] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < nw; ++k) {
      const int c = s_w[k];
      s_w[k] = tot;
      tot += c;
    }
    s_w[16] = tot ? atomicAdd(n, tot) : 0;
  }
  __syncthreads();
  if (pred) list[s_w[16] + s_w[w] + __popcll(b & lanemask_lt())] = value;
  __syncthreads();
}

__global__ __launch_bounds__(kPushBlock) void k_cell_candidates(const int* __restrict__ cell_start,
                                                                const int* __restrict__ num_cells, int min_pts,
                                                                CloudParams cp, int* __restrict__ cand,
                                                                int* __restrict__ num_cand,
                                                                uint8_t* __restrict__ dense) {
  __shared__ int s_w[17];
  const int nc = *num_cells;
  // every thread of a workgroup runs the same trip count (block_push synchronises)
  for (int base = blockIdx.x * kPushBlock; base < nc; base += gridDim.x * kPushBlock) {
    const int c = base + static_cast<int>(threadIdx.x);
    bool cand_c = false;
    if (c < nc) {
      const int cnt = cell_start[c + 1] - cell_start[c];
      dense[c] = 0;
      cand_c = cnt >= cell_minpts(cp, cell_start[c], min_pts);
    }
    block_push(cand, num_cand, cand_c, c, s_w);
  }
}

// Tight box per candidate cell by a reduction over G lanes, then the guard. Two
// launches share the candidate list: G = 64 (a wavefront per cell) takes the cells
// of more than kSmallCell points, G = 8 (eight cells per wavefront) the others, so
// a batch's many small cells do not each hold a whole wavefront.
constexpr int kSmallCell = 64;

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

__global__ __launch_bounds__(kBlock) void k_prim_flags(const int* __restrict__ cell_id,
                                                       const int* __restrict__ cell_start,
                                                       const uint8_t* __restrict__ dense, int64_t n,
                                                       int* __restrict__ pflag) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    int c = cell_id[i];
    pflag[i] = (!dense[c] || cell_start[c] == i) ? 1 : 0;
  }
}

// pidx holds the exclusive scan of pflag: the primitive index of every point
// that opens a primitive (a point outside dense cells, or a dense cell's first).
template <int D>
__global__ __launch_bounds__(kPushBlock) void k_prims(KeyIn keys, const float* __restrict__ xs, int64_t n,
                                                  const int* __restrict__ cell_id, const int* __restrict__ cell_start,
                                                  const uint8_t* __restrict__ dense, const float4* __restrict__ cell_lo,
                                                  const float4* __restrict__ cell_hi, const int* __restrict__ pidx,
                                                  int* __restrict__ prim_start,
                                                  int* __restrict__ prim_cnt, float4* __restrict__ prim_lo,
                                                  float4* __restrict__ prim_hi, uint64_t* __restrict__ prim_key,
                                                  int* __restrict__ dense_list, int* __restrict__ num_dense,
                                                  int* __restrict__ labels, uint8_t* __restrict__ core) {
  __shared__ int s_w[17];
  const bool wide = keys.wide();
  // Every thread of a workgroup runs the same trip count and reaches the one
  // block_push call of each trip (it synchronises the workgroup).
  for (int64_t base = blockIdx.x * int64_t(kPushBlock); base < n; base += int64_t(gridDim.x) * kPushBlock) {
    const int64_t i64 = base + threadIdx.x;
    bool opens_dense = false;
    int pd = 0;
    if (i64 < n) {
      const int i = static_cast<int>(i64);
      const int c = cell_id[i];
      const int s = cell_start[c];
      opens_dense = dense[c] && i == s;
      if (dense[c]) {
        const int p = pidx[s];
        labels[i] = s;
        core[i] = 1;
        if (opens_dense) {
          const float4 cl = cell_lo[c];
          prim_start[p] = s;
          prim_cnt[p] = -(cell_start[c + 1] - s);
          prim_lo[p] = make_float4(cl.x, cl.y, cl.z, __int_as_float(-2 - s));
          prim_hi[p] = cell_hi[c];
          prim_key[p] = key_at(keys, wide, i);
          pd = p;
        }
      } else {
        const int p = pidx[i];  // a point primitive: its box is the point
        labels[i] = i;
        core[i] = 0;
        prim_start[p] = i;
        prim_cnt[p] = 1;
        prim_lo[p] = make_float4(xs[i], xs[n + i], D == 3 ? xs[2 * n + i] : 0.0f, __int_as_float(i));
        prim_key[p] = key_at(keys, wide, i);
      }
    }
    block_push(dense_list, num_dense, opens_dense, pd, s_w);
  }
}

inline int grid_for(int64_t n) {
  int64_t g = ceil_div(n, kBlock * 4);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

void cells_t(const KeyIn& keys, int64_t n, int dim, const float* xs, float eps2, int min_pts, int* cell_id,
             int* cell_start, int* cand, uint8_t* dense, float4* cell_lo, float4* cell_hi, int* pflag,
             int* prim_start, int* prim_cnt, float4* prim_lo, float4* prim_hi, uint64_t* prim_key, int* dense_list,
             int* labels, uint8_t* core, int* misc, int* bsums, int64_t scan_blocks, const CloudParams& cp,
             hipStream_t s) {
  int* d_cells = misc + kMiscNumCells;
  int* d_cand = misc + kMiscNumCand;
  int* d_prims = misc + kMiscNumPrims;
  int* d_dense = misc + kMiscNumDense;
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_cell_heads, dim3(g), dim3(kBlock), 0, s, keys, n, pflag);
  device_scan(pflag, cell_id, n, nullptr, bsums, scan_blocks, d_cells, s);
  hipLaunchKernelGGL(k_cell_start, dim3(g), dim3(kBlock), 0, s, pflag, n, cell_id, cell_start, d_cells);
  fill_u32(reinterpret_cast<uint32_t*>(d_cand), 0, 1, s);
  const int gp = static_cast<int>(std::min<int64_t>(ceil_div(n, kPushBlock), 65536));
  hipLaunchKernelGGL(k_cell_candidates, dim3(gp), dim3(kPushBlock), 0, s, cell_start, d_cells, min_pts, cp, cand,
                     d_cand, dense);
  const int gb = 2048;  // 8192 wavefronts, grid-stride over candidate cells
  if (dim == 3) {
    hipLaunchKernelGGL((k_cell_boxes<3, 64>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, cand, d_cand, eps2, cp,
                       dense, cell_lo, cell_hi);
    hipLaunchKernelGGL((k_cell_boxes<3, 8>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, cand, d_cand, eps2, cp,
                       dense, cell_lo, cell_hi);
  } else {
    hipLaunchKernelGGL((k_cell_boxes<2, 64>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, cand, d_cand, eps2, cp,
                       dense, cell_lo, cell_hi);
    hipLaunchKernelGGL((k_cell_boxes<2, 8>), dim3(gb), dim3(kBlock), 0, s, xs, n, cell_start, cand, d_cand, eps2, cp,
                       dense, cell_lo, cell_hi);
  }
  hipLaunchKernelGGL(k_prim_flags, dim3(g), dim3(kBlock), 0, s, cell_id, cell_start, dense, n, pflag);
  int* pidx = cand;  // candidates are no longer needed; reuse for primitive indices
  device_scan(pflag, pidx, n, nullptr, bsums, scan_blocks, d_prims, s);
  if (dim == 3)
    hipLaunchKernelGGL((k_prims<3>), dim3(gp), dim3(kPushBlock), 0, s, keys, xs, n, cell_id, cell_start, dense,
                       cell_lo, cell_hi, pidx, prim_start, prim_cnt, prim_lo, prim_hi, prim_key, dense_list,
                       d_dense, labels, core);
  else
    hipLaunchKernelGGL((k_prims<2>), dim3(gp), dim3(kPushBlock), 0, s, keys, xs, n, cell_id, cell_start, dense,
                       cell_lo, cell_hi, pidx, prim_start, prim_cnt, prim_lo, prim_hi, prim_key, dense_list,
                       d_dense, labels, core);
}

}  // namespace

void densebox_cells(const void* sorted_keys, bool key64, const int* d_key64, int64_t n, int dim, const float* xs,
                    float eps2, int min_pts, int* cell_id, int* cell_start, int* cand, uint8_t* cell_dense,
                    float4* cell_lo, float4* cell_hi, int* pflag, int* prim_start, int* prim_cnt, float4* prim_lo,
                    float4* prim_hi, uint64_t* prim_key, int* dense_list, int* labels, uint8_t* core, int* misc,
                    int* bsums, int64_t scan_blocks, hipStream_t s, int key_shift, const int* cl_minpts,
                    const float* cl_eps2) {
  // per-cloud parameters come with batches, whose keys are always 64-bit
  CloudParams cp{static_cast<const uint64_t*>(sorted_keys), key_shift, cl_minpts, cl_eps2};
  const KeyIn keys{sorted_keys, d_key64, key64 ? 1 : 0};
  cells_t(keys, n, dim, xs, eps2, min_pts, cell_id, cell_start, cand, cell_dense, cell_lo, cell_hi, pflag, prim_start,
          prim_cnt, prim_lo, prim_hi, prim_key, dense_list, labels, core, misc, bsums, scan_blocks, cp, s);
}

}  // namespace fdb
