// Preparation kernels: scene bounds and finite check, space-filling-curve keys
// (Section 4.1 orders queries and primitives along a Morton curve), grid-cell
// keys for DenseBox (Section 4.2), and the gather of points into sorted SoA.
#include "fdb_device.hpp"
#include "fdb_internal.hpp"
#include "fdbscan.h"

namespace fdb {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int per_block, int cap = 65536) {
  int64_t g = ceil_div(n, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, uint8_t v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Workgroup reduction of per-thread axis bounds, then one atomic per axis.
// bounds[0..2] hold lo, bounds[4..6] hi, as order-preserving uints (pre-filled
// with 0xffffffff / 0).
template <int D>
__device__ __forceinline__ void bounds_reduce(float* lo, float* hi, bool bad, uint32_t* __restrict__ bounds,
                                              uint32_t* __restrict__ info) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
    }
  }
  __shared__ float s_lo[kBlock / 64][3], s_hi[kBlock / 64][3];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (bad) s_bad = 1;
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      s_lo[w][k] = lo[k];
      s_hi[w][k] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < D) {
    int k = threadIdx.x;
    float a = s_lo[0][k], b = s_hi[0][k];
    for (int j = 1; j < kBlock / 64; ++j) {
      a = fminf(a, s_lo[j][k]);
      b = fmaxf(b, s_hi[j][k]);
    }
    if (a <= b) {  // this block saw at least one finite value on axis k
      atomicMin(bounds + k, f2ord(a));
      atomicMax(bounds + 4 + k, f2ord(b));
    }
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(info, FDB_INFO_NONFINITE);
}

// min/max per axis over all points; flags non-finite coordinates (any layout).
template <int D>
__global__ __launch_bounds__(kBlock) void k_bounds(const float* __restrict__ pts, int64_t n,
                                                   uint32_t* __restrict__ bounds, uint32_t* __restrict__ info) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      float v = pts[i * D + k];
      bad |= !isfinite(v);
      lo[k] = fminf(lo[k], v);
      hi[k] = fmaxf(hi[k], v);
    }
  }
  bounds_reduce<D>(lo, hi, bad, bounds, info);
}

// Same over the coordinates as one flat float array read 16 bytes at a time
// (pts 16-byte aligned). The grid stride is a multiple of D, so every chunk a
// thread reads starts on the same axis: lane j of its float4s always holds
// axis (4 c0 + j) mod D, and four running min/max pairs suffice.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bounds_v4(const float* __restrict__ pts, int64_t nflat,
                                                      uint32_t* __restrict__ bounds, uint32_t* __restrict__ info) {
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(pts);
  const int64_t nch = nflat >> 2;
  const int64_t T = int64_t(gridDim.x) * kBlock;
  const int64_t c0 = blockIdx.x * int64_t(kBlock) + threadIdx.x;
  float l4[4] = {INFINITY, INFINITY, INFINITY, INFINITY}, h4[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  auto take = [&](float4 v) {
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bad |= !isfinite(e[j]);
      l4[j] = fminf(l4[j], e[j]);
      h4[j] = fmaxf(h4[j], e[j]);
    }
  };
  int64_t c = c0;
  for (; c + 7 * T < nch; c += 8 * T) {  // eight 16-byte loads in flight per lane
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p4[c + u * T];
#pragma unroll
    for (int u = 0; u < 8; ++u) take(v[u]);
  }
  for (; c < nch; c += T) take(p4[c]);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = static_cast<int>((4 * c0 + j) % D);
#pragma unroll
    for (int kk = 0; kk < D; ++kk)
      if (k == kk) {
        lo[kk] = fminf(lo[kk], l4[j]);
        hi[kk] = fmaxf(hi[kk], h4[j]);
      }
  }
  if (c0 == 0) {  // the last nflat mod 4 coordinates
    for (int64_t e = nch * 4; e < nflat; ++e) {
      const float v = pts[e];
      const int k = static_cast<int>(e % D);
      bad |= !isfinite(v);
#pragma unroll
      for (int kk = 0; kk < D; ++kk)
        if (k == kk) {
          lo[kk] = fminf(lo[kk], v);
          hi[kk] = fmaxf(hi[kk], v);
        }
    }
  }
  bounds_reduce<D>(lo, hi, bad, bounds, info);
}

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

// 63-bit (3D, 21 bits per axis) or 62-bit (2D, 31 bits per axis) Morton codes
// of the points normalised to the scene bounds, and the identity permutation.
template <int D>
__global__ __launch_bounds__(kBlock) void k_morton(const float* __restrict__ pts, int64_t n,
                                                   const uint32_t* __restrict__ bounds, uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals, int passes,
                                                   uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8 * 256];
  hist_clear(s_h, passes);
  constexpr uint32_t maxq = D == 3 ? 0x1fffffu : 0x7fffffffu;
  float lo[D], scale[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    lo[k] = ord2f(bounds[k]);
    float ext = ord2f(bounds[4 + k]) - lo[k];
    scale[k] = ext > 0.0f ? static_cast<float>(maxq) / ext : 0.0f;
  }
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    uint64_t code;
    if constexpr (D == 3) {
      code = (spread3(quantize(pts[i * 3 + 0], lo[0], scale[0], maxq)) << 2) |
             (spread3(quantize(pts[i * 3 + 1], lo[1], scale[1], maxq)) << 1) |
             spread3(quantize(pts[i * 3 + 2], lo[2], scale[2], maxq));
    } else {
      code = (spread2(quantize(pts[i * 2 + 0], lo[0], scale[0], maxq)) << 1) |
             spread2(quantize(pts[i * 2 + 1], lo[1], scale[1], maxq));
    }
    keys[i] = code;
    vals[i] = static_cast<uint32_t>(i);
    hist_add(code, true, passes, s_h);
  }
  hist_flush(s_h, passes, hist);
}

// The DenseBox grid of one cloud (Section 4.2: cells of side h = eps/sqrt(d)),
// sized here from the bounds so that nothing returns to the host mid-call. The
// side is shrunk by 2^-20 so that rounding in the cell index rarely pushes a
// cell's extent past h (the exactness guard catches the rest). A grid wider than
// a 64-bit key holds gets wider cells (every pair in a dense cell still passes the
// guard). The isolated-point test runs for 32-bit keys when its occupancy map (one
// bit per cell, a 64-bit word per brick of 64 cells) fits in map_bytes and its
// brick table (a bit per brick) in n 32-bit words.
template <int D>
__global__ void k_grid_plan(const uint32_t* __restrict__ bounds, float eps, int64_t n, int64_t map_bytes,
                            GridPlan* __restrict__ plan, uint32_t* __restrict__ info) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  constexpr int maxbits = D == 3 ? 21 : 31;
  const double side0 = static_cast<double>(eps) / sqrt(static_cast<double>(D)) * (1.0 - 1.0 / 1048576.0);
  double ext[3] = {0.0, 0.0, 0.0}, emax = 0.0;
  for (int k = 0; k < D; ++k) {
    const double e = static_cast<double>(ord2f(bounds[4 + k])) - static_cast<double>(ord2f(bounds[k]));
    ext[k] = e >= 0.0 && e <= 3.0e38 ? e : 0.0;  // an empty or non-finite extent: one cell
    emax = ext[k] > emax ? ext[k] : emax;
  }
  const double top = static_cast<double>((1u << maxbits) - 2u);  // at most 2^maxbits - 1 cells per axis
  double side = side0;
  int coarse = 0;
  if (!(side > 0.0) || !(emax / side < top)) {
    side = emax > 0.0 ? emax / top : 1.0;
    side = side > side0 ? side : side0;
    coarse = 1;
  }
  const float ih = static_cast<float>(1.0 / side);
  int bits = 0;
  GridPlan g;
  for (int k = 0; k < 4; ++k) {
    g.inv_h[k] = k < D ? ih : 0.0f;
    uint32_t c = 1;
    if (k < D) {
      const double cells = floor(ext[k] / side) + 1.0;
      c = cells < top + 1.0 ? static_cast<uint32_t>(cells) : static_cast<uint32_t>(top + 1.0);
    }
    g.ncell[k] = c;
    int b = 0;
    while ((uint64_t(1) << b) < c) ++b;
    bits = b > bits ? b : bits;
  }
  g.bits = bits;
  g.key64 = D * bits > 32 ? 1 : 0;
  g.passes = (D * bits + 7) / 8;
  g.start = (g.passes & 1) ? 0 : 1;
  g.coarse = coarse;
  // isolated-point test: a word per brick of 64 grid cells (in map_bytes) and a
  // table bit per brick (in an n-int buffer); reach = eps / side in cell units plus
  // a slack for the rounding of the cell coordinates t = (x - lo) * inv_h: each is
  // within 2^-23 t of exact, so a difference within cmax 2^-22 (times 4 here), and
  // the fp32 test passes pairs up to eps (1 + 2^-22) apart (2^-16 here)
  double cmax = 1.0;
  for (int k = 0; k < D; ++k) cmax = g.ncell[k] > cmax ? g.ncell[k] : cmax;
  const double reach = static_cast<double>(eps) * static_cast<double>(ih) * (1.0 + 1.0 / 65536.0) +
                       4.0 * (cmax / 4194304.0 + 1.0 / 1048576.0) + 1.0 / 65536.0;
  g.lone_words = D * bits >= 6 ? int64_t(1) << (D * bits - 6) : 1;
  g.reach = static_cast<float>(reach);
  g.lone_on = (!g.key64 && bits >= 1 && reach < 1.999 && g.lone_words * 8 <= map_bytes &&
               (g.lone_words + 63) / 64 * 2 <= n) ? 1 : 0;
  *plan = g;
  if (coarse) atomicOr(info, FDB_INFO_DENSEBOX_FALLBACK);
}

constexpr int kGridKeyItems = 4;

// DenseBox cell keys: cell c_k = floor((x_k - lo_k) / h), clamped to the grid; the
// key is the Morton interleave of the cell coordinates, so equal keys are one cell
// and cells follow the curve. Written as 32- or 64-bit words as the plan says, into
// the buffer the plan names, with the identity permutation beside them.
template <int D>
__global__ __launch_bounds__(kBlock) void k_gridkeys(const float* __restrict__ pts, int64_t n,
                                                     const uint32_t* __restrict__ bounds,
                                                     const GridPlan* __restrict__ plan, void* __restrict__ keys0,
                                                     void* __restrict__ keys1, uint32_t* __restrict__ vals0,
                                                     uint32_t* __restrict__ vals1, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8 * 256];
  const GridPlan g = *plan;
  const int passes = g.passes;
  hist_clear(s_h, passes);
  uint32_t* vals = g.start ? vals1 : vals0;
  void* keys = g.start ? keys1 : keys0;
  float lo[D];
#pragma unroll
  for (int k = 0; k < D; ++k) lo[k] = ord2f(bounds[k]);
  // kGridKeyItems points per thread and trip, their loads issued together
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i0 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i0 < n; i0 += kGridKeyItems * stride) {
    float x[kGridKeyItems][D];
#pragma unroll
    for (int t = 0; t < kGridKeyItems; ++t) {
      const int64_t i = i0 + t * stride;
#pragma unroll
      for (int k = 0; k < D; ++k) x[t][k] = i < n ? pts[i * D + k] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < kGridKeyItems; ++t) {
      const int64_t i = i0 + t * stride;
      const bool valid = i < n;
      uint32_t c[D];
#pragma unroll
      for (int k = 0; k < D; ++k) c[k] = quantize(x[t][k], lo[k], g.inv_h[k], g.ncell[k] - 1);
      uint64_t code;
      if constexpr (D == 3)
        code = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
      else
        code = (spread2(c[0]) << 1) | spread2(c[1]);
      if (valid) {
        if (g.key64)
          static_cast<uint64_t*>(keys)[i] = code;
        else
          static_cast<uint32_t*>(keys)[i] = static_cast<uint32_t>(code);
        if (passes == 0) vals[i] = static_cast<uint32_t>(i);  // else the first sort pass makes them
      }
      hist_add(code, valid, passes, s_h);
    }
  }
  hist_flush(s_h, passes, hist);
}

// Gather points into key order, structure-of-arrays. The reads are random 12-byte
// rows, so each thread first loads kPermItems indices, then issues all of their
// row loads before any store: several gathers in flight per lane instead of one.
constexpr int kPermItems = 4;

template <int D>
__global__ __launch_bounds__(kBlock) void k_permute(const float* __restrict__ pts, int64_t n,
                                                    const uint32_t* __restrict__ perm, float* __restrict__ xs,
                                                    uint32_t* __restrict__ info) {
  const int64_t stride = int64_t(gridDim.x) * kBlock * kPermItems;
  for (int64_t base = blockIdx.x * int64_t(kBlock) * kPermItems + threadIdx.x; base < n; base += stride) {
    int64_t o[kPermItems];
#pragma unroll
    for (int t = 0; t < kPermItems; ++t) {
      const int64_t i = base + t * kBlock;
      o[t] = i < n ? static_cast<int64_t>(perm[i]) : 0;
    }
    float v[kPermItems][D];
#pragma unroll
    for (int t = 0; t < kPermItems; ++t) {
      if (o[t] >= n) {
        atomicOr(info, kInternalBit);
        o[t] = 0;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) v[t][k] = pts[o[t] * D + k];
    }
#pragma unroll
    for (int t = 0; t < kPermItems; ++t) {
      const int64_t i = base + t * kBlock;
      if (i < n) {
#pragma unroll
        for (int k = 0; k < D; ++k) xs[k * n + i] = v[t][k];
      }
    }
  }
}

}  // namespace

// Several fills in one launch: element t of the concatenated segments.
__global__ void k_fill_multi(FillList L) {
  int64_t total = 0;
  for (int k = 0; k < L.count; ++k) total += L.seg[k].n;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    int64_t r = t;
    int k = 0;
    while (r >= L.seg[k].n) r -= L.seg[k++].n;
    L.seg[k].p[r] = L.seg[k].v;
  }
}

void fill_multi(const FillList& L, hipStream_t s) {
  int64_t total = 0;
  for (int k = 0; k < L.count; ++k) total += L.seg[k].n;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_fill_multi, dim3(grid_for(total, kBlock * 4)), dim3(kBlock), 0, s, L);
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kBlock * 4)), dim3(kBlock), 0, s, p, v, n);
}

void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, kBlock * 16)), dim3(kBlock), 0, s, p, v, n);
}

void launch_bounds(const float* pts, int64_t n, int dim, uint32_t* bounds, uint32_t* info, hipStream_t s) {
  if ((reinterpret_cast<uintptr_t>(pts) & 15) == 0) {
    const int64_t nflat = n * dim;
    // few workgroups (each ends with one atomic per axis bound on shared words)
    int g = grid_for(ceil_div(nflat, 4), kBlock * 8, 768);
    g = (g + dim - 1) / dim * dim;  // grid stride a multiple of dim
    if (dim == 3)
      hipLaunchKernelGGL(k_bounds_v4<3>, dim3(g), dim3(kBlock), 0, s, pts, nflat, bounds, info);
    else
      hipLaunchKernelGGL(k_bounds_v4<2>, dim3(g), dim3(kBlock), 0, s, pts, nflat, bounds, info);
    return;
  }
  int g = grid_for(n, kBlock * 16, 2048);
  if (dim == 3)
    hipLaunchKernelGGL(k_bounds<3>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, info);
  else
    hipLaunchKernelGGL(k_bounds<2>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, info);
}

void launch_morton(const float* pts, int64_t n, int dim, const uint32_t* bounds, uint64_t* keys, uint32_t* vals,
                   int sort_bits, uint32_t* hist, hipStream_t s) {
  const int passes = (sort_bits + 7) / 8;
  fill_u32(hist, 0, passes * 256, s);
  int g = grid_for(n, kBlock * 16, 1024);  // a workgroup histogram per 4096+ keys, flushes kept few
  if (dim == 3)
    hipLaunchKernelGGL(k_morton<3>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, keys, vals, passes, hist);
  else
    hipLaunchKernelGGL(k_morton<2>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, keys, vals, passes, hist);
}

void launch_grid_plan(const uint32_t* bounds, int dim, float eps, int64_t n, int64_t map_bytes, GridPlan* plan,
                      uint32_t* info, hipStream_t s) {
  if (dim == 3)
    hipLaunchKernelGGL(k_grid_plan<3>, dim3(1), dim3(64), 0, s, bounds, eps, n, map_bytes, plan, info);
  else
    hipLaunchKernelGGL(k_grid_plan<2>, dim3(1), dim3(64), 0, s, bounds, eps, n, map_bytes, plan, info);
}

void launch_gridkeys(const float* pts, int64_t n, int dim, const uint32_t* bounds, const GridPlan* plan,
                     void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, uint32_t* hist, hipStream_t s,
                     bool hist_clear) {
  if (hist_clear) fill_u32(hist, 0, 8 * 256, s);
  // A workgroup histogram per 4096+ keys, at most 1024 of them: each flushes up to 2048 bins into the
  // one global histogram, and fewer flushes contend less at L2 than more workgroups gain.
  int g = grid_for(n, kBlock * 16, 1024);
  if (dim == 3)
    hipLaunchKernelGGL(k_gridkeys<3>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, plan, keys0, keys1, vals0, vals1,
                       hist);
  else
    hipLaunchKernelGGL(k_gridkeys<2>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, plan, keys0, keys1, vals0, vals1,
                       hist);
}

void launch_permute(const float* pts, int64_t n, int dim, const uint32_t* perm, float* xs, uint32_t* info,
                    hipStream_t s) {
  int g = grid_for(n, kBlock * kPermItems);
  if (dim == 3)
    hipLaunchKernelGGL(k_permute<3>, dim3(g), dim3(kBlock), 0, s, pts, n, perm, xs, info);
  else
    hipLaunchKernelGGL(k_permute<2>, dim3(g), dim3(kBlock), 0, s, pts, n, perm, xs, info);
}

}  // namespace fdb
