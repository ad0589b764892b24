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
  for (; c + 3 * T < nch; c += 4 * T) {
    const float4 a = p4[c], b = p4[c + T], d = p4[c + 2 * T], f = p4[c + 3 * T];
    take(a);
    take(b);
    take(d);
    take(f);
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

// DenseBox grid (Section 4.2): cell c_k = floor((x_k - lo_k) / h), h = eps/sqrt(d)
// (inv_h supplied slightly above sqrt(d)/eps), clamped to the grid; the key is
// the Morton interleave of the cell coordinates, so equal keys are one cell and
// cells follow the curve.
template <int D, typename K>
__global__ __launch_bounds__(kBlock) void k_gridkeys(const float* __restrict__ pts, int64_t n,
                                                     const uint32_t* __restrict__ bounds, float ihx, float ihy,
                                                     float ihz, uint32_t ncx, uint32_t ncy, uint32_t ncz,
                                                     K* __restrict__ keys, uint32_t* __restrict__ vals, int passes,
                                                     uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8 * 256];
  hist_clear(s_h, passes);
  const float ih[3] = {ihx, ihy, ihz};
  const uint32_t nc[3] = {ncx, ncy, ncz};
  float lo[D];
#pragma unroll
  for (int k = 0; k < D; ++k) lo[k] = ord2f(bounds[k]);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    uint32_t c[D];
#pragma unroll
    for (int k = 0; k < D; ++k) c[k] = quantize(pts[i * D + k], lo[k], ih[k], nc[k] - 1);
    uint64_t code;
    if constexpr (D == 3)
      code = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
    else
      code = (spread2(c[0]) << 1) | spread2(c[1]);
    keys[i] = static_cast<K>(code);
    vals[i] = static_cast<uint32_t>(i);
    hist_add(static_cast<K>(code), true, passes, s_h);
  }
  hist_flush(s_h, passes, hist);
}

// Gather points into Morton order, structure-of-arrays.
template <int D>
__global__ __launch_bounds__(kBlock) void k_permute(const float* __restrict__ pts, int64_t n,
                                                    const uint32_t* __restrict__ perm, float* __restrict__ xs,
                                                    uint32_t* __restrict__ info) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    int64_t o = perm[i];
    if (o >= n) {
      atomicOr(info, kInternalBit);
      o = 0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) xs[k * n + i] = pts[o * D + k];
  }
}

}  // namespace

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
  int g = grid_for(n, kBlock * 16, 2048);  // a workgroup histogram per 4096+ keys
  if (dim == 3)
    hipLaunchKernelGGL(k_morton<3>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, keys, vals, passes, hist);
  else
    hipLaunchKernelGGL(k_morton<2>, dim3(g), dim3(kBlock), 0, s, pts, n, bounds, keys, vals, passes, hist);
}

void launch_gridkeys(const float* pts, int64_t n, int dim, const uint32_t* bounds, const float* ih,
                     const uint32_t* nc, int bits, bool key64, void* keys, uint32_t* vals, int sort_bits,
                     uint32_t* hist, hipStream_t s) {
  (void)bits;
  const int passes = (sort_bits + 7) / 8;
  fill_u32(hist, 0, passes * 256, s);
  int g = grid_for(n, kBlock * 16, 2048);  // a workgroup histogram per 4096+ keys
  if (dim == 3) {
    if (key64)
      hipLaunchKernelGGL((k_gridkeys<3, uint64_t>), dim3(g), dim3(kBlock), 0, s, pts, n, bounds, ih[0], ih[1],
                         ih[2], nc[0], nc[1], nc[2], static_cast<uint64_t*>(keys), vals, passes, hist);
    else
      hipLaunchKernelGGL((k_gridkeys<3, uint32_t>), dim3(g), dim3(kBlock), 0, s, pts, n, bounds, ih[0], ih[1],
                         ih[2], nc[0], nc[1], nc[2], static_cast<uint32_t*>(keys), vals, passes, hist);
  } else {
    if (key64)
      hipLaunchKernelGGL((k_gridkeys<2, uint64_t>), dim3(g), dim3(kBlock), 0, s, pts, n, bounds, ih[0], ih[1],
                         0.0f, nc[0], nc[1], 1u, static_cast<uint64_t*>(keys), vals, passes, hist);
    else
      hipLaunchKernelGGL((k_gridkeys<2, uint32_t>), dim3(g), dim3(kBlock), 0, s, pts, n, bounds, ih[0], ih[1],
                         0.0f, nc[0], nc[1], 1u, static_cast<uint32_t*>(keys), vals, passes, hist);
  }
}

void launch_permute(const float* pts, int64_t n, int dim, const uint32_t* perm, float* xs, uint32_t* info,
                    hipStream_t s) {
  int g = grid_for(n, kBlock * 4);
  if (dim == 3)
    hipLaunchKernelGGL(k_permute<3>, dim3(g), dim3(kBlock), 0, s, pts, n, perm, xs, info);
  else
    hipLaunchKernelGGL(k_permute<2>, dim3(g), dim3(kBlock), 0, s, pts, n, perm, xs, info);
}

}  // namespace fdb
