// Batches of independent point clouds in one launch sequence. Every cloud keeps
// its own eps and minPts; the result per cloud is the one a separate call
// would give. Keys put the cloud id above the Morton bits, so one sort orders
// all clouds and, in Karras' hierarchy, the points (or DenseBox primitives) of
// one cloud - all keys sharing that prefix - form exactly one subtree: the node
// whose range is the cloud's range, which is internal node first or last of
// that range (a Karras node's index is one end of its range), or a leaf.
#include "fdb_device.hpp"
#include "fdb_internal.hpp"
#include "fdbscan.h"

namespace fdb {

namespace {

constexpr int kBlock = 256;
constexpr int kCloudNonfinite = 1, kCloudBadParams = 2, kCloudBadRange = 4;

__device__ __forceinline__ uint64_t spread3(uint32_t v) {  // 21 bits -> every third bit of 63
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x001f00000000ffffull;
  x = (x | x << 16) & 0x001f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint64_t spread2(uint32_t v) {  // 32 bits -> every other bit of 64
  uint64_t x = v;
  x = (x | x << 16) & 0x0000ffff0000ffffull;
  x = (x | x << 8) & 0x00ff00ff00ff00ffull;
  x = (x | x << 4) & 0x0f0f0f0f0f0f0f0full;
  x = (x | x << 2) & 0x3333333333333333ull;
  x = (x | x << 1) & 0x5555555555555555ull;
  return x;
}

__device__ __forceinline__ uint32_t quantize(float v, float lo, float scale, uint32_t maxq) {
  float t = fmaxf((v - lo) * scale, 0.0f);
  float fmax = static_cast<float>(maxq);
  return t >= fmax ? maxq : static_cast<uint32_t>(t);
}

// Cloud c's range, clamped into [0, n] (offsets come from the caller's device
// memory and cannot be checked on the host without waiting).
__device__ __forceinline__ void cloud_range(const int64_t* off, int c, int64_t n, int64_t& b, int64_t& e) {
  b = off[c];
  e = off[c + 1];
  b = b < 0 ? 0 : (b > n ? n : b);
  e = e < b ? b : (e > n ? n : e);
}

// Largest cloud c in [lo, hi] with off[c] <= i (binary search; with offsets out
// of order the answer is still some cloud in [lo, hi]).
__device__ __forceinline__ int cloud_at(const int64_t* __restrict__ off, int64_t i, int lo, int hi) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Points are processed in chunks of kChunk consecutive points per workgroup
// (kItems per thread, striped); a chunk's clouds are [s_c[0], s_c[1]].
constexpr int kItems = 16;
constexpr int kChunk = kBlock * kItems;

__device__ __forceinline__ void chunk_clouds(const int64_t* off, int num_clouds, int64_t base, int64_t n, int* s_c) {
  if (threadIdx.x == 0) {
    const int64_t last = (base + kChunk < n ? base + kChunk : n) - 1;
    const int c0 = cloud_at(off, base, 0, num_clouds - 1);
    s_c[0] = c0;
    s_c[1] = cloud_at(off, last, c0, num_clouds - 1);
  }
  __syncthreads();
}

// Per-cloud bounds (order-preserving uints: cl_ord[8c + k] lo, [8c + 4 + k] hi,
// pre-filled with 0xffffffff / 0) and non-finite flags, one chunk per
// workgroup: a workgroup reduction for each cloud the chunk touches, then one
// atomic per axis bound.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cloud_bounds(const float* __restrict__ pts, const int64_t* __restrict__ off,
                                                         int num_clouds, int64_t n, uint32_t* __restrict__ cl_ord,
                                                         int* __restrict__ cl_flags) {
  __shared__ int s_c[2];
  __shared__ float s_r[kBlock / 64][6];
  __shared__ int s_bad[kBlock / 64];
  const int64_t base = blockIdx.x * int64_t(kChunk);
  chunk_clouds(off, num_clouds, base, n, s_c);
  const int c0 = s_c[0], c1 = s_c[1];
  int cl[kItems];
  float v[kItems][3];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    cl[k] = i < n ? (c0 == c1 ? c0 : cloud_at(off, i, c0, c1)) : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) v[k][d] = (i < n && d < D) ? pts[i * D + d] : 0.0f;
  }
  const int w = threadIdx.x >> 6;
  for (int c = c0; c <= c1; ++c) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if (cl[k] == c)
#pragma unroll
        for (int d = 0; d < D; ++d) {
          bad |= !isfinite(v[k][d]);
          lo[d] = fminf(lo[d], v[k][d]);
          hi[d] = fmaxf(hi[d], v[k][d]);
        }
#pragma unroll
    for (int d = 0; d < D; ++d)
      for (int o = 32; o > 0; o >>= 1) {
        lo[d] = fminf(lo[d], __shfl_xor(lo[d], o));
        hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], o));
      }
    bad = ballot(bad != 0) ? 1 : 0;
    if ((threadIdx.x & 63) == 0) {
      for (int d = 0; d < 3; ++d) {
        s_r[w][d] = lo[d];
        s_r[w][3 + d] = hi[d];
      }
      s_bad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int b = 0;
      for (int j = 0; j < kBlock / 64; ++j) {
        b |= s_bad[j];
        for (int d = 0; d < D; ++d) {
          lo[d] = fminf(lo[d], s_r[j][d]);
          hi[d] = fmaxf(hi[d], s_r[j][3 + d]);
        }
      }
      for (int d = 0; d < D; ++d)
        if (lo[d] <= hi[d]) {  // some finite value of this cloud in the chunk
          atomicMin(cl_ord + 8 * c + d, f2ord(lo[d]));
          atomicMax(cl_ord + 8 * c + 4 + d, f2ord(hi[d]));
        }
      if (b) atomicOr(cl_flags + c, kCloudNonfinite);
    }
    __syncthreads();
  }
}

// Per-cloud validity, eps^2, minPts and key scale (points normalised to the
// cloud's box, or DenseBox cells of side eps/sqrt(d), slightly shrunk; the
// exactness guard covers any rounding). One thread per cloud.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cloud_params(const int64_t* __restrict__ off, int num_clouds, int64_t n,
                                                         const float* __restrict__ eps, const int32_t* __restrict__ mp,
                                                         int bpd, int densebox, const uint32_t* __restrict__ cl_ord,
                                                         float4* __restrict__ cl_lo, float4* __restrict__ cl_scale,
                                                         float* __restrict__ cl_eps2, int* __restrict__ cl_minpts,
                                                         int* __restrict__ cl_flags, uint32_t* __restrict__ info) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= num_clouds) return;
  int64_t b, e;
  cloud_range(off, c, n, b, e);
  int flags = cl_flags[c];
  if (off[c] != b || off[c + 1] != e || (c == 0 && b != 0) || (c == num_clouds - 1 && e != n)) flags |= kCloudBadRange;
  const float ec = eps[c];
  const int mc = mp[c];
  if (!(ec > 0.0f) || !isfinite(ec) || mc < 1) flags |= kCloudBadParams;
  cl_flags[c] = flags;
  if (flags & kCloudNonfinite) atomicOr(info, FDB_INFO_NONFINITE);
  if (flags & (kCloudBadParams | kCloudBadRange)) atomicOr(info, FDB_INFO_BAD_PARAMS);
  cl_eps2[c] = ec * ec;
  cl_minpts[c] = mc;
  const uint32_t maxq = (1u << bpd) - 1u;
  float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f}, sc[3] = {0.0f, 0.0f, 0.0f};
  for (int k = 0; k < D; ++k) {
    lo[k] = ord2f(cl_ord[8 * c + k]);
    hi[k] = ord2f(cl_ord[8 * c + 4 + k]);
    if (!(lo[k] <= hi[k])) lo[k] = hi[k] = 0.0f;  // empty cloud
    if (densebox) {
      const double side = static_cast<double>(ec) / sqrt(static_cast<double>(D)) * (1.0 - 1.0 / 1048576.0);
      sc[k] = side > 0.0 ? static_cast<float>(1.0 / side) : 0.0f;
    } else {
      const float ext = hi[k] - lo[k];
      sc[k] = ext > 0.0f ? static_cast<float>(maxq) / ext : 0.0f;
    }
  }
  cl_lo[c] = make_float4(lo[0], lo[1], lo[2], 0.0f);
  cl_scale[c] = make_float4(sc[0], sc[1], sc[2], 0.0f);
}

// Lower-bound words of every cloud start at the largest order-preserving value.
__global__ __launch_bounds__(kBlock) void k_ord_init(uint32_t* __restrict__ cl_ord, int num_clouds) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= num_clouds) return;
  for (int k = 0; k < 4; ++k) cl_ord[8 * c + k] = 0xffffffffu;
}

// Keys (cloud id << shift | Morton of the point's, or its cell's, coordinates),
// the identity permutation, and the radix sort's digit counts; one chunk of
// consecutive points per workgroup.
template <int D>
__global__ __launch_bounds__(kBlock) void k_batch_keys(const float* __restrict__ pts, const int64_t* __restrict__ off,
                                                       int num_clouds, int64_t n, const float4* __restrict__ cl_lo,
                                                       const float4* __restrict__ cl_scale, int bpd, int shift,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       int passes, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8 * 256];
  __shared__ int s_c[2];
  hist_clear(s_h, passes);
  const int64_t base = blockIdx.x * int64_t(kChunk);
  chunk_clouds(off, num_clouds, base, n, s_c);
  const int c0 = s_c[0], c1 = s_c[1];
  const uint32_t maxq = (1u << bpd) - 1u;
#pragma unroll 4
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int c = valid ? (c0 == c1 ? c0 : cloud_at(off, i, c0, c1)) : c0;
    const float4 lo4 = cl_lo[c], sc4 = cl_scale[c];
    const float lo[3] = {lo4.x, lo4.y, lo4.z}, sc[3] = {sc4.x, sc4.y, sc4.z};
    uint64_t key = 0;
    if (valid) {
      uint32_t q[D];
#pragma unroll
      for (int d = 0; d < D; ++d) q[d] = quantize(pts[i * D + d], lo[d], sc[d], maxq);
      uint64_t code;
      if constexpr (D == 3)
        code = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
      else
        code = (spread2(q[0]) << 1) | spread2(q[1]);
      key = (static_cast<uint64_t>(c) << shift) | code;
      keys[i] = key;
      vals[i] = static_cast<uint32_t>(i);
    }
    hist_add(key, valid, passes, s_h);
  }
  hist_flush(s_h, passes, hist);
}

// Subtree of each cloud: its primitive range [a, b] and the node covering it.
// FDbscan primitives are points (the range is the cloud's own); DenseBox
// primitive ranges come from the primitive index of each cloud's first point
// (a cloud's first point always opens a primitive: cells never span clouds).
__global__ __launch_bounds__(kBlock) void k_cloud_roots(const int64_t* __restrict__ off, int num_clouds, int64_t n,
                                                        const int* __restrict__ pidx, const int* __restrict__ d_m,
                                                        const int* __restrict__ other, int* __restrict__ root,
                                                        int* __restrict__ end, uint32_t* __restrict__ info) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= num_clouds) return;
  int64_t b, e;
  cloud_range(off, c, n, b, e);
  if (e <= b) {  // empty cloud: no queries ever reach it
    root[c] = static_cast<int>(kEnd);
    end[c] = -1;
    return;
  }
  int pa, pb;
  if (pidx) {
    const int m = *d_m;
    pa = pidx[b];
    pb = e < n ? pidx[e] - 1 : m - 1;
  } else {
    pa = static_cast<int>(b);
    pb = static_cast<int>(e - 1);
  }
  end[c] = pb;
  if (pa == pb) {
    root[c] = static_cast<int>(kLeaf | static_cast<uint32_t>(pa));
  } else if (other[pa] == pb) {
    root[c] = pa;
  } else if (other[pb] == pa) {
    root[c] = pb;
  } else {
    atomicOr(info, kInternalBit);
    root[c] = static_cast<int>(kEnd);
  }
}

// Per-cloud cluster ids: a cluster's global id is the number of cluster
// leaders (smallest core input index of a cluster) at smaller input indices, so
// a cloud's ids are that count minus the count at the cloud's first input
// index, and its K the difference across the cloud.

__global__ __launch_bounds__(kBlock) void k_batch_cluster_ids(const int* __restrict__ labels,
                                                              const uint8_t* __restrict__ core,
                                                              const int* __restrict__ minorig,
                                                              const uint32_t* __restrict__ bits,
                                                              const int* __restrict__ wpre,
                                                              const uint64_t* __restrict__ pkeys, int shift,
                                                              const int64_t* __restrict__ off, int num_clouds,
                                                              int64_t n, const int* __restrict__ total,
                                                              int* __restrict__ cid) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    if (!(core[i] && labels[i] == i)) continue;
    const int c = min(static_cast<int>(pkeys[i] >> shift), num_clouds - 1);
    int64_t b, e;
    cloud_range(off, c, n, b, e);
    cid[i] = leaders_before(bits, wpre, minorig[i], n, total) - leaders_before(bits, wpre, b, n, total);
  }
}

// K per cloud, or -1 where the cloud's labels are undefined (a coordinate that
// is not finite, eps or minPts out of range, offsets out of order).
__global__ __launch_bounds__(kBlock) void k_batch_counts(const uint32_t* __restrict__ bits,
                                                         const int* __restrict__ wpre, const int64_t* __restrict__ off,
                                                         int num_clouds, int64_t n, const int* __restrict__ total,
                                                         const int* __restrict__ cl_flags,
                                                         int32_t* __restrict__ num_clusters) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= num_clouds) return;
  int64_t b, e;
  cloud_range(off, c, n, b, e);
  num_clusters[c] =
      cl_flags[c] ? -1 : leaders_before(bits, wpre, e, n, total) - leaders_before(bits, wpre, b, n, total);
}

inline int grid_for(int64_t n) {
  int64_t g = ceil_div(n, kBlock * 4);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

}  // namespace

void batch_prep(const float* pts, const int64_t* off, int num_clouds, int64_t n, int dim, const float* eps,
                const int32_t* min_pts, int bpd, bool densebox, uint32_t* cl_ord, float4* cl_lo, float4* cl_scale,
                float* cl_eps2, int* cl_minpts, int* cl_flags, uint32_t* info, hipStream_t s) {
  fill_u32(cl_ord, 0u, 8 * int64_t(num_clouds), s);  // hi words 0; k_ord_init sets the lo words
  hipLaunchKernelGGL(k_ord_init, dim3(static_cast<unsigned>(ceil_div(num_clouds, kBlock))), dim3(kBlock), 0, s,
                     cl_ord, num_clouds);
  fill_u32(reinterpret_cast<uint32_t*>(cl_flags), 0u, num_clouds, s);
  const unsigned chunks = static_cast<unsigned>(ceil_div(n, kChunk));
  const unsigned pg = static_cast<unsigned>(ceil_div(num_clouds, kBlock));
  if (dim == 3) {
    if (chunks) hipLaunchKernelGGL(k_cloud_bounds<3>, dim3(chunks), dim3(kBlock), 0, s, pts, off, num_clouds, n, cl_ord,
                                   cl_flags);
    hipLaunchKernelGGL(k_cloud_params<3>, dim3(pg), dim3(kBlock), 0, s, off, num_clouds, n, eps, min_pts, bpd,
                       densebox ? 1 : 0, cl_ord, cl_lo, cl_scale, cl_eps2, cl_minpts, cl_flags, info);
  } else {
    if (chunks) hipLaunchKernelGGL(k_cloud_bounds<2>, dim3(chunks), dim3(kBlock), 0, s, pts, off, num_clouds, n, cl_ord,
                                   cl_flags);
    hipLaunchKernelGGL(k_cloud_params<2>, dim3(pg), dim3(kBlock), 0, s, off, num_clouds, n, eps, min_pts, bpd,
                       densebox ? 1 : 0, cl_ord, cl_lo, cl_scale, cl_eps2, cl_minpts, cl_flags, info);
  }
}

void batch_keys(const float* pts, const int64_t* off, int num_clouds, int64_t n, int dim, const float4* cl_lo,
                const float4* cl_scale, int bpd, int shift, uint64_t* keys, uint32_t* vals, int sort_bits,
                uint32_t* hist, hipStream_t s) {
  const int passes = (sort_bits + 7) / 8;
  fill_u32(hist, 0, passes * 256, s);
  const unsigned chunks = static_cast<unsigned>(ceil_div(n, kChunk));
  if (!chunks) return;
  if (dim == 3)
    hipLaunchKernelGGL(k_batch_keys<3>, dim3(chunks), dim3(kBlock), 0, s, pts, off, num_clouds, n, cl_lo, cl_scale,
                       bpd, shift, keys, vals, passes, hist);
  else
    hipLaunchKernelGGL(k_batch_keys<2>, dim3(chunks), dim3(kBlock), 0, s, pts, off, num_clouds, n, cl_lo, cl_scale,
                       bpd, shift, keys, vals, passes, hist);
}

void batch_roots(const int64_t* off, int num_clouds, int64_t n, const int* pidx, const int* d_m, const int* other,
                 int* root, int* end, uint32_t* info, hipStream_t s) {
  hipLaunchKernelGGL(k_cloud_roots, dim3(static_cast<unsigned>(ceil_div(num_clouds, kBlock))), dim3(kBlock), 0, s,
                     off, num_clouds, n, pidx, d_m, other, root, end, info);
}

void batch_cluster_ids(const int* labels, const uint8_t* core, const int* minorig, const uint32_t* bits,
                       const int* wpre, const uint64_t* pkeys, int shift, const int64_t* off, int num_clouds,
                       int64_t n, const int* total, const int* cl_flags, int* cid, int32_t* num_clusters,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_batch_cluster_ids, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, minorig, bits, wpre,
                     pkeys, shift, off, num_clouds, n, total, cid);
  if (num_clusters)
    hipLaunchKernelGGL(k_batch_counts, dim3(static_cast<unsigned>(ceil_div(num_clouds, kBlock))), dim3(kBlock), 0, s,
                       bits, wpre, off, num_clouds, n, total, cl_flags, num_clusters);
}

}  // namespace fdb
