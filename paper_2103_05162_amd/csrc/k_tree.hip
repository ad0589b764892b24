// Linear BVH over m primitives sorted by Morton key (Section 4.1 uses an LBVH
// in the manner of Karras 2012): one thread per internal node finds its leaf
// range and split from the longest common prefix of neighbouring keys (equal
// keys compare by index), a second pass writes the escape links ("ropes") for
// stack-less traversal, and a bottom-up pass computes exact min/max boxes.
#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

constexpr int kBlock = 256;

// Common-prefix length of keys i and j; -1 outside [0, m). Equal keys are told
// apart by their positions, so every prefix is strictly ordered.
template <typename K>
__device__ __forceinline__ int prefix_len(const K* __restrict__ keys, int m, int i, int64_t j) {
  if (j < 0 || j >= m) return -1;
  K a = keys[i], b = keys[j];
  if (a == b) return int(8 * sizeof(K)) + __clz(static_cast<uint32_t>(i) ^ static_cast<uint32_t>(j));
  if constexpr (sizeof(K) == 8)
    return __clzll(static_cast<unsigned long long>(a ^ b));
  else
    return __clz(static_cast<uint32_t>(a ^ b));
}

// Internal node i: its range is [min(i,j), max(i,j)] and its split gamma
// separates [first, gamma] from [gamma+1, last]. Children are internal node
// gamma / gamma+1, or leaves when their side holds one primitive.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_karras(const K* __restrict__ keys, int m_cap, const int* __restrict__ d_m,
                                                   int* __restrict__ other, int* __restrict__ gamma_out,
                                                   int* __restrict__ parent, int* __restrict__ flags) {
  const int m = d_m ? *d_m : m_cap;
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= m - 1) return;
  int dl = prefix_len(keys, m, i, int64_t(i) - 1);
  int dr = prefix_len(keys, m, i, int64_t(i) + 1);
  int d = dr > dl ? 1 : -1;
  int dmin = dr > dl ? dl : dr;
  int64_t lmax = 2;
  while (prefix_len(keys, m, i, i + lmax * d) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (prefix_len(keys, m, i, i + (l + t) * d) > dmin) l += t;
  int64_t j = i + l * d;
  int dnode = prefix_len(keys, m, i, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (prefix_len(keys, m, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int g = static_cast<int>(i + s * d + (d < 0 ? -1 : 0));
  int first = static_cast<int>(d > 0 ? i : j), last = static_cast<int>(d > 0 ? j : i);
  other[i] = static_cast<int>(j);
  gamma_out[i] = g;
  flags[i] = 0;  // the refit's arrival counter of node i
  // parent[] holds internal nodes at [0, m-1) and leaf l at m-1+l
  parent[first == g ? (m - 1) + g : g] = i;
  parent[last == g + 1 ? (m - 1) + g + 1 : g + 1] = i;
  if (i == 0) parent[0] = -1;
}

// Pre-order successor of a subtree whose last leaf is l: the right child of the
// node splitting l from l+1, which is internal node l+1 when that node's range
// starts at l+1 and leaf l+1 otherwise.
__device__ __forceinline__ int successor(const int* __restrict__ other, int m, int l) {
  if (l >= m - 1) return static_cast<int>(kEnd);
  int r = l + 1;
  if (r <= m - 2 && other[r] > r) return r;
  return static_cast<int>(kLeaf | static_cast<uint32_t>(r));
}

__global__ __launch_bounds__(kBlock) void k_ropes(const int* __restrict__ other, int m_cap, const int* __restrict__ d_m,
                                                  int* __restrict__ rope, int* __restrict__ leaf_rope) {
  const int m = d_m ? *d_m : m_cap;
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < m - 1) {
    int last = other[i] > i ? other[i] : i;
    rope[i] = successor(other, m, last);
  }
  if (i < m) leaf_rope[i] = successor(other, m, i);
}

struct Box {
  float lo[3], hi[3];
};

// Leaves are points (FDbscan: leaf l is sorted point l), or DenseBox
// primitives: a dense cell's stored box, or the single point it starts at.
// DenseBox leaves: primitive l's record lo[l] holds a single point and its
// sorted index (w >= 0), or a dense cell's low corner (w < 0; the high corner
// is hi[l]).
struct LeafSrc {
  const float4* lo;  // null: leaves are the sorted points
  const float4* hi;
};

template <int D>
__device__ __forceinline__ Box leaf_box(int l, const float* __restrict__ xs, int64_t n, const LeafSrc& ls) {
  Box b;
  if (ls.lo) {
    const float4 a = ls.lo[l];
    b.lo[0] = a.x; b.lo[1] = a.y; b.lo[2] = a.z;
    if (__float_as_int(a.w) < 0) {
      const float4 c = ls.hi[l];
      b.hi[0] = c.x; b.hi[1] = c.y; b.hi[2] = c.z;
    } else {
      b.hi[0] = a.x; b.hi[1] = a.y; b.hi[2] = a.z;
    }
    return b;
  }
  b.lo[0] = b.hi[0] = xs[l];
  b.lo[1] = b.hi[1] = xs[n + l];
  b.lo[2] = b.hi[2] = D == 3 ? xs[2 * n + l] : 0.0f;
  return b;
}

// Node boxes cross workgroups (and XCDs) inside the refit kernel, so they are
// written and read with agent-scope (L2-bypassing) 64-bit atomics; a writer
// drains its stores (s_waitcnt vmcnt(0)) before it bumps the arrival counter,
// and the second arriver only reads after that counter's value came back. No
// L2-wide writeback or invalidate is needed.
__device__ __forceinline__ uint64_t pack2(float a, float b) {
  return uint64_t(__float_as_uint(a)) | (uint64_t(__float_as_uint(b)) << 32);
}
__device__ __forceinline__ float lo32(uint64_t v) { return __uint_as_float(static_cast<uint32_t>(v)); }
__device__ __forceinline__ float hi32(uint64_t v) { return __uint_as_float(static_cast<uint32_t>(v >> 32)); }

__device__ __forceinline__ void store_node(float4* node_a, float4* node_b, int p, const Box& b, int o, int g) {
  uint64_t* a = reinterpret_cast<uint64_t*>(node_a + kNodeStride * size_t(p));
  uint64_t* c = reinterpret_cast<uint64_t*>(node_b + kNodeStride * size_t(p));
  st_agent64(a, pack2(b.lo[0], b.lo[1]));
  st_agent64(a + 1, pack2(b.lo[2], __int_as_float(o)));
  st_agent64(c, pack2(b.hi[0], b.hi[1]));
  st_agent64(c + 1, pack2(b.hi[2], __int_as_float(g)));
}

__device__ __forceinline__ Box load_node(const float4* node_a, const float4* node_b, int k) {
  const uint64_t* a = reinterpret_cast<const uint64_t*>(node_a + kNodeStride * size_t(k));
  const uint64_t* c = reinterpret_cast<const uint64_t*>(node_b + kNodeStride * size_t(k));
  uint64_t a0 = ld_agent64(a), a1 = ld_agent64(a + 1), c0 = ld_agent64(c), c1 = ld_agent64(c + 1);
  Box b;
  b.lo[0] = lo32(a0); b.lo[1] = hi32(a0); b.lo[2] = lo32(a1);
  b.hi[0] = lo32(c0); b.hi[1] = hi32(c0); b.hi[2] = lo32(c1);
  return b;
}

// The same accesses as 128-bit buffer instructions with the same cache policy
// (sc1, as the agent-scope 64-bit accesses above): a node is 32 contiguous
// bytes, so it takes two stores or loads instead of four. Buffer offsets are
// 32-bit, so this serves node arrays below 2 GiB (kRefitBufMaxNodes).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kPolicySc1 = 16;                  // buffer cache-policy operand: sc1
constexpr uint32_t kBufferWord3 = 0x00020000u;  // raw-buffer descriptor word 3 on gfx9 parts
constexpr int64_t kRefitBufMaxNodes = ((int64_t(1) << 31) - 1) / (16 * kNodeStride);

__device__ __forceinline__ void store_node_buf(__amdgpu_buffer_rsrc_t r, int p, const Box& b, int o, int g) {
  const u32x4 va = {__float_as_uint(b.lo[0]), __float_as_uint(b.lo[1]), __float_as_uint(b.lo[2]),
                    static_cast<uint32_t>(o)};
  const u32x4 vb = {__float_as_uint(b.hi[0]), __float_as_uint(b.hi[1]), __float_as_uint(b.hi[2]),
                    static_cast<uint32_t>(g)};
  __builtin_amdgcn_raw_buffer_store_b128(va, r, p * (16 * kNodeStride), 0, kPolicySc1);
  __builtin_amdgcn_raw_buffer_store_b128(vb, r, p * (16 * kNodeStride) + 16, 0, kPolicySc1);
}

__device__ __forceinline__ Box load_node_buf(__amdgpu_buffer_rsrc_t r, int k) {
  const u32x4 va = __builtin_amdgcn_raw_buffer_load_b128(r, k * (16 * kNodeStride), 0, kPolicySc1);
  const u32x4 vb = __builtin_amdgcn_raw_buffer_load_b128(r, k * (16 * kNodeStride) + 16, 0, kPolicySc1);
  Box b;
  b.lo[0] = __uint_as_float(va.x); b.lo[1] = __uint_as_float(va.y); b.lo[2] = __uint_as_float(va.z);
  b.hi[0] = __uint_as_float(vb.x); b.hi[1] = __uint_as_float(vb.y); b.hi[2] = __uint_as_float(vb.z);
  return b;
}

// Bottom-up refit: each leaf walks towards the root; at every internal node the
// second of the two arriving threads merges its box with the sibling's and
// continues upwards, so every box is the exact min/max of its leaves. A node
// whose leaves all belong to this workgroup's kRefitBlock (its index then lies among
// them too) is met in LDS: each arriver leaves its box in the slot of its side
// and counts itself with a workgroup-scope atomic. Only nodes spanning
// workgroups take the device-scope protocol, so most arrivals never leave the CU.
constexpr int kRefitBlock = 256;  // leaves per workgroup of the refit

template <int D, bool BUF>
__global__ __launch_bounds__(kRefitBlock) void k_refit(int m_cap, const int* __restrict__ d_m, const float* __restrict__ xs,
                                                  int64_t n,
                                                  LeafSrc ls, const int* __restrict__ other, const int* __restrict__ gamma,
                                                  const int* __restrict__ parent, int* __restrict__ flags,
                                                  float4* node_a, float4* node_b, uint32_t* __restrict__ info) {
  __shared__ int s_arrive[kRefitBlock];
  __shared__ float s_side[2][6][kRefitBlock];  // [child side][lo.xyz, hi.xyz][node - first leaf]
  const int m = d_m ? *d_m : m_cap;
  const int L0 = blockIdx.x * kRefitBlock;
  if (m < 2 || L0 >= m) return;  // whole workgroup
  s_arrive[threadIdx.x] = 0;
  __syncthreads();
  const int L1 = min(L0 + kRefitBlock, m) - 1;  // this workgroup's leaves are [L0, L1]
  const int l = L0 + static_cast<int>(threadIdx.x);
  if (l >= m) return;
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(node_a, 0, BUF ? m_cap * (16 * kNodeStride) : 0, kBufferWord3);
  Box box = leaf_box<D>(l, xs, n, ls);
  int prev = l;
  bool prev_leaf = true;
  int p = parent[(m - 1) + l];
  while (p >= 0) {
    if (p >= m - 1) {
      atomicOr(info, kInternalBit);
      return;
    }
    const int o = other[p], g = gamma[p];
    const int first = o < p ? o : p, last = o > p ? o : p;
    if (first < 0 || last >= m || g < first || g >= last) {
      atomicOr(info, kInternalBit);
      return;
    }
    const bool left_leaf = first == g, right_leaf = last == g + 1;
    const bool came_left = prev == g && prev_leaf == left_leaf;
    Box sib;
    if (first >= L0 && last <= L1) {
      const int slot = p - L0, side = came_left ? 0 : 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s_side[side][k][slot] = box.lo[k];
        s_side[side][3 + k][slot] = box.hi[k];
      }
      if (__hip_atomic_fetch_add(&s_arrive[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) return;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sib.lo[k] = s_side[side ^ 1][k][slot];
        sib.hi[k] = s_side[side ^ 1][3 + k][slot];
      }
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's node stores have landed
      if (atomicAdd(flags + p, 1) == 0) return;
      if (came_left)
        sib = right_leaf ? leaf_box<D>(g + 1, xs, n, ls)
                         : (BUF ? load_node_buf(rb, g + 1) : load_node(node_a, node_b, g + 1));
      else
        sib = left_leaf ? leaf_box<D>(g, xs, n, ls) : (BUF ? load_node_buf(rb, g) : load_node(node_a, node_b, g));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      box.lo[k] = fminf(box.lo[k], sib.lo[k]);
      box.hi[k] = fmaxf(box.hi[k], sib.hi[k]);
    }
    if (BUF)
      store_node_buf(rb, p, box, o, g);
    else
      store_node(node_a, node_b, p, box, o, g);
    prev = p;
    prev_leaf = false;
    p = parent[p];
  }
}

// m_cap: number of primitives, or an upper bound when d_m (device) holds it.
template <typename K>
void build_t(const K* keys, int m_cap, const int* d_m, int dim, const float* xs, int64_t n_pts,
             const LeafSrc& ls, float4* node_a, float4* node_b, int* rope,
             int* leaf_rope, int* parent, int* flags, int* other, int* gamma, uint32_t* info, hipStream_t s) {
  if (m_cap <= 0) return;
  int g = static_cast<int>(ceil_div(m_cap, kBlock));
  if (m_cap >= 2) {
    hipLaunchKernelGGL(k_karras<K>, dim3(g), dim3(kBlock), 0, s, keys, m_cap, d_m, other, gamma, parent, flags);
  }
  hipLaunchKernelGGL(k_ropes, dim3(g), dim3(kBlock), 0, s, other, m_cap, d_m, rope, leaf_rope);
  if (m_cap >= 2) {
    const bool buf = m_cap <= kRefitBufMaxNodes;
    const dim3 rg(static_cast<unsigned>(ceil_div(m_cap, kRefitBlock))), rb(kRefitBlock);
    if (dim == 3 && buf)
      hipLaunchKernelGGL((k_refit<3, true>), rg, rb, 0, s, m_cap, d_m, xs, n_pts, ls, other, gamma, parent, flags,
                         node_a, node_b, info);
    else if (dim == 3)
      hipLaunchKernelGGL((k_refit<3, false>), rg, rb, 0, s, m_cap, d_m, xs, n_pts, ls, other, gamma, parent, flags,
                         node_a, node_b, info);
    else if (buf)
      hipLaunchKernelGGL((k_refit<2, true>), rg, rb, 0, s, m_cap, d_m, xs, n_pts, ls, other, gamma, parent, flags,
                         node_a, node_b, info);
    else
      hipLaunchKernelGGL((k_refit<2, false>), rg, rb, 0, s, m_cap, d_m, xs, n_pts, ls, other, gamma, parent, flags,
                         node_a, node_b, info);
  }
}

}  // namespace

void build_lbvh(const void* keys, bool key64, int m, int dim, const float* xs, int64_t n_pts, const float4* prim_lo,
                const float4* prim_hi, float4* node_a, float4* node_b, int* rope, int* leaf_rope, int* parent,
                int* flags, int* other, int* gamma, const int* d_m, uint32_t* info, hipStream_t s) {
  const LeafSrc ls{prim_lo, prim_hi};
  if (key64)
    build_t(static_cast<const uint64_t*>(keys), m, d_m, dim, xs, n_pts, ls, node_a, node_b, rope, leaf_rope, parent,
            flags, other, gamma, info, s);
  else
    build_t(static_cast<const uint32_t*>(keys), m, d_m, dim, xs, n_pts, ls, node_a, node_b, rope, leaf_rope, parent,
            flags, other, gamma, info, s);
}

}  // namespace fdb
