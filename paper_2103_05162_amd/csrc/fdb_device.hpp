// Device-side building blocks shared by the FDbscan / FDbscan-DenseBox kernels:
// the fp32 neighbour test, the conservative box test, the lock-free union-find
// and a few wavefront helpers. gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdb {

// ---- node references -------------------------------------------------------
// Internal node k of an m-primitive LBVH is referenced by k (0..m-2); leaf l by
// l | kLeaf; kEnd terminates a rope walk. m is capped at 2^30.
constexpr uint32_t kLeaf = 0x80000000u;
constexpr uint32_t kEnd = 0x7fffffffu;

// ---- the neighbour test ----------------------------------------------------
// dist(x,y) <= eps (Section 2.1) evaluated as s <= fl32(eps*eps) with
// s = (dx*dx + dy*dy) + dz*dz, every operation rounded on its own. The library is
// compiled with -ffp-contract=off so no product is fused into an add; the same
// order is used everywhere the test or a bound on it is computed.
template <int D>
__device__ __forceinline__ float dist2(const float* p, float qx, float qy, float qz) {
  float dx = p[0] - qx;
  float dy = p[1] - qy;
  float s = dx * dx;
  float t = dy * dy;
  s = s + t;
  if constexpr (D == 3) {
    float dz = p[2] - qz;
    float u = dz * dz;
    s = s + u;
  }
  return s;
}

template <int D>
__device__ __forceinline__ float dist2v(float px, float py, float pz, float qx, float qy, float qz) {
  float dx = px - qx;
  float dy = py - qy;
  float s = dx * dx;
  float t = dy * dy;
  s = s + t;
  if constexpr (D == 3) {
    float dz = pz - qz;
    float u = dz * dz;
    s = s + u;
  }
  return s;
}

// Lower bound of dist2 between query q and any point of box [lo,hi], computed in
// the same rounding order: per axis the gap g = max(lo-q, q-hi, 0) (rounded
// subtraction is monotone, so g <= |fl(p-q)| for every p in the box), then the
// same sum of squares. Entering a node iff this bound <= eps2 therefore never
// skips a pair that passes the neighbour test.
template <int D>
__device__ __forceinline__ float box_dist2(float qx, float qy, float qz, float lx, float ly, float lz,
                                           float hx, float hy, float hz) {
  float gx = fmaxf(fmaxf(lx - qx, qx - hx), 0.0f);
  float gy = fmaxf(fmaxf(ly - qy, qy - hy), 0.0f);
  float s = gx * gx;
  float t = gy * gy;
  s = s + t;
  if constexpr (D == 3) {
    float gz = fmaxf(fmaxf(lz - qz, qz - hz), 0.0f);
    float u = gz * gz;
    s = s + u;
  }
  return s;
}

// Same bound between two boxes (every point of box A against every point of box B).
template <int D>
__device__ __forceinline__ float boxbox_dist2(const float* alo, const float* ahi, float lx, float ly, float lz,
                                              float hx, float hy, float hz) {
  float gx = fmaxf(fmaxf(lx - ahi[0], alo[0] - hx), 0.0f);
  float gy = fmaxf(fmaxf(ly - ahi[1], alo[1] - hy), 0.0f);
  float s = gx * gx;
  float t = gy * gy;
  s = s + t;
  if constexpr (D == 3) {
    float gz = fmaxf(fmaxf(lz - ahi[2], alo[2] - hz), 0.0f);
    float u = gz * gz;
    s = s + u;
  }
  return s;
}

// ---- agent-scope atomics -----------------------------------------------------
// On gfx950 each XCD has its own L2; agent-scope atomic loads and stores bypass it
// (sc1), so values written by a workgroup on another XCD are seen within the
// same kernel. Used for every access whose freshness matters for progress.
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int cas_agent(int* p, int expected, int desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found (== expected on success)
}
__device__ __forceinline__ uint64_t ld_agent64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- union-find on the flat labels array (Sections 3.1, 4.3) -----------------
// labels[x] is x's parent; a root points to itself. Unions hook the larger root
// under the smaller with one compare-and-swap, so among core points a parent
// never exceeds its child and the root of a set is its smallest member. Find
// uses path halving ("intermediate pointer jumping"): each visited node is
// re-pointed at its grandparent. A stale parent read is always an ancestor, so
// the re-pointing is safe under concurrency.
// Walks are capped: a cycle or a runaway walk (impossible unless something else
// is broken) raises kInternalBit in *info and stops instead of spinning forever.
constexpr uint32_t kInternalBit = 4u;  // FDB_INFO_INTERNAL
constexpr uint32_t kForestBit = 32u;   // FDB_INFO_FOREST
constexpr int kWalkCap = 1 << 22;

__device__ __forceinline__ int uf_find(int* labels, int x, uint32_t* info) {
  int p = ld_agent(labels + x);
  for (int it = 0; p != x; ++it) {
    int g = ld_agent(labels + p);
    if (g == p) return p;
    st_agent(labels + x, g);
    x = g;
    p = ld_agent(labels + x);
    if (it > kWalkCap) {
      atomicOr(info, kInternalBit);
      break;
    }
  }
  return x;
}

// Merge the sets of a and b; returns a root of the merged set at the time of
// the merge (a valid short-circuit key afterwards: sets only ever grow).
__device__ __forceinline__ int uf_union(int* labels, int a, int b, uint32_t* info) {
  for (int it = 0;; ++it) {
    if (it > kWalkCap) {
      atomicOr(info, kInternalBit);
      return a;
    }
    a = uf_find(labels, a, info);
    b = uf_find(labels, b, info);
    if (a == b) return a;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    // a > b: hook a under b
    int seen = cas_agent(labels + a, a, b);
    if (seen == a) return b;
    a = seen;  // a was hooked meanwhile; continue from its new parent
  }
}

// Border claim (Section 3.2): a non-core point y joins the cluster of a core
// point x only if nobody claimed it yet; labels[y] == y marks "not a member".
// One compare-and-swap replaces the critical section, so y is never a hook
// target and cannot bridge two clusters.
__device__ __forceinline__ void uf_claim(int* labels, int y, int x) { (void)cas_agent(labels + y, y, x); }

// ---- order-preserving float <-> uint (for atomic min/max of floats) ----------
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// ---- XCD-aware workgroup order -------------------------------------------------
// gfx950 hands workgroups to its 8 XCDs round-robin (workgroup b runs on XCD
// b % 8), and each XCD has its own L2. Renumbering so that XCD x gets one
// contiguous range of logical workgroups keeps Morton-neighbouring queries -
// which walk the same subtrees - on the same L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b % kNumXcd, k = b / kNumXcd;
  const int per = nb / kNumXcd, rem = nb % kNumXcd;
  return x * per + (x < rem ? x : rem) + k;
}

// Index of thread `tid` of workgroup b (of blocks of `bdim` threads) when the
// active range [0, m) is split into 8 contiguous chunks, one per XCD (chunks are
// whole workgroups); -1 for threads past their chunk. A grid of
// 8 * ceil(ceil(n/8)/bdim) workgroups, for any n >= m, covers [0, m).
__device__ __forceinline__ int64_t xcd_spread(int b, int bdim, int tid, int64_t m) {
  const int64_t chunk = ((m + kNumXcd - 1) / kNumXcd + bdim - 1) / bdim * bdim;
  const int64_t off = static_cast<int64_t>(b / kNumXcd) * bdim;
  if (off >= chunk) return -1;
  return (b % kNumXcd) * chunk + off + tid;
}

// ---- canonical ids --------------------------------------------------------------
// Cluster leaders are kept as one bit per input index (bits[o >> 5], bit o & 31);
// wpre[w] is the number of leaders in words before w. The number of leaders at
// input indices below x (x <= n) is then one load, one popcount and one add.
__device__ __forceinline__ int leaders_before(const uint32_t* __restrict__ bits, const int* __restrict__ wpre,
                                              int64_t x, int64_t n, const int* __restrict__ total) {
  if (x >= n) return *total;
  const int r = static_cast<int>(x & 31);
  return wpre[x >> 5] + __popc(bits[x >> 5] & ((1u << r) - 1u));
}

// ---- wavefront helpers ---------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ---- radix-sort digit histograms ---------------------------------------------
// Lanes of the wavefront whose 8-bit digit d equals this lane's, among lanes
// with `valid`.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    bool bit = (d >> b) & 1u;
    uint64_t bb = ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Count the 8-bit digits of `key` (passes from the least significant) into the
// workgroup's histograms s_h[p * 256 + digit]. A digit shared by every counted
// lane (typical of a key's high digits) costs one LDS atomic; otherwise each
// lane adds its own (same-address lanes serialise in LDS). Lanes outside the
// wavefront's active set do not count.
template <typename K>
__device__ __forceinline__ void hist_add(K key, bool valid, int passes, uint32_t* s_h) {
  const uint64_t vm = ballot(valid);
  if (!vm) return;
  const int first = __ffsll(static_cast<unsigned long long>(vm)) - 1;
  for (int p = 0; p < passes; ++p) {
    const uint32_t d = static_cast<uint32_t>(key >> (8 * p)) & 0xffu;
    const uint32_t d0 = static_cast<uint32_t>(__shfl(static_cast<int>(d), first));
    if (!ballot(valid && d != d0)) {
      if (lane_id() == first) atomicAdd(s_h + p * 256 + d0, static_cast<uint32_t>(__popcll(vm)));
    } else if (valid) {
      atomicAdd(s_h + p * 256 + d, 1u);
    }
  }
}

// Workgroup histogram lifecycle around hist_add: clear, then add to the global
// counts (only non-zero bins). Every thread of the workgroup must call both.
__device__ __forceinline__ void hist_clear(uint32_t* s_h, int passes) {
  for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) s_h[i] = 0;
  __syncthreads();
}
__device__ __forceinline__ void hist_flush(const uint32_t* s_h, int passes, uint32_t* hist) {
  __syncthreads();
  for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) {
    const uint32_t v = s_h[i];
    if (v) atomicAdd(hist + i, v);
  }
}

}  // namespace fdb
