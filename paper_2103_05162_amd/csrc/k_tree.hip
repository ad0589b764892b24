// Linear BVH over m primitives sorted by Morton key (Section 4.1 uses an LBVH
// in the manner of Karras 2012). The hierarchy is Karras' binary radix tree over
// the keys (equal keys compare by index), numbered as Karras numbers it, but it is
// built bottom-up in the same pass that computes the exact min/max boxes (the
// agglomerative order of Apetrei 2014): every leaf climbs, a node merges with the
// neighbour across its more similar edge, and the second of two arrivers at a
// split carries the merged node on. A second pass writes the escape links
// ("ropes") for stack-less traversal.
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

// Bottom-up build and refit. Node [i, j] (i < j) of Karras' tree has the split
// where the common prefix of neighbouring keys is shortest inside it; its parent
// adds the neighbour across the edge (i-1 | i or j | j+1) with the longer common
// prefix, and that edge is the parent's split. Karras' numbering follows: a left
// child [i, s] is node s, a right child [s+1, j] is node s+1, and the root is 0.
// Each leaf climbs: at split s the two children meet, the second arriver learns
// the other's far end and box, writes the parent (range end, split, box) at the
// parent's own index once it knows on which side the parent hangs, and goes on.
//
// A meeting whose parent lies within this workgroup's kRefitBlock leaves is held
// in LDS (box in the slot of the arriver's side, far end by an atomic exchange).
// Both arrivers decide that alike from the prefix lengths of the workgroup's
// leaves: a left child [i, s] inside the workgroup has its sibling end inside it
// exactly when some edge in (s, L1] is less similar than s, which a suffix
// minimum over the workgroup's edges answers; a right child likewise with a
// prefix minimum. Other meetings exchange the far end through ends[s] (cleared
// to -1 beforehand) with one device-scope atomic exchange, after the first
// arriver's node stores have drained; node records are written and read with
// agent-scope (L2-bypassing) accesses, since the sibling may run on another XCD.
constexpr int kRefitBlock = 256;  // leaves per workgroup of the build

// Common-prefix length of edge k (keys k and k+1); -1 for the edges before the
// first and after the last key, which are less similar than every inner edge.
template <typename K>
__device__ __forceinline__ int edge_len(const K* __restrict__ keys, int m, int64_t k) {
  return k < 0 || k >= m - 1 ? -1 : prefix_len(keys, m, static_cast<int>(k), k + 1);
}

__device__ __forceinline__ void cut_add(float4* cut, int* cut_n, uint32_t ref, int last, const Box& b) {
  const int k = atomicAdd(cut_n, 1);
  if (k >= kCutMax) return;  // too many: the walks then ignore the cut
  cut[2 * k] = make_float4(b.lo[0], b.lo[1], b.lo[2], __uint_as_float(ref));
  cut[2 * k + 1] = make_float4(b.hi[0], b.hi[1], b.hi[2], __int_as_float(last));
}

template <typename K, int D, bool BUF>
__global__ __launch_bounds__(kRefitBlock) void k_build_up(const K* __restrict__ keys, int m_cap,
                                                     const int* __restrict__ d_m, const float* __restrict__ xs,
                                                     int64_t n, LeafSrc ls, int* __restrict__ other,
                                                     int* __restrict__ gamma, int* __restrict__ ends, float4* node_a,
                                                     float4* node_b, uint32_t* __restrict__ info,
                                                     float4* __restrict__ cut, int* __restrict__ cut_n, int cut_div) {
  constexpr int E = kRefitBlock + 1;  // edges L0-1 .. L0+255
  __shared__ int s_far[kRefitBlock];
  __shared__ float s_side[2][6][kRefitBlock];  // [child side][lo.xyz, hi.xyz][split - L0]
  __shared__ int s_pmin[E], s_smin[E], s_len[E];
  const int m = d_m ? *d_m : m_cap;
  const int L0 = blockIdx.x * kRefitBlock;
  if (m < 2 || L0 >= m) return;  // whole workgroup
  const int L1 = min(L0 + kRefitBlock, m) - 1;  // this workgroup's leaves are [L0, L1]
  const int t = threadIdx.x;
  const int ne = L1 - L0 + 2;  // edges L0-1 .. L1, entry e is edge L0-1+e
  s_far[t] = -1;
  for (int e = t; e < ne; e += kRefitBlock) s_len[e] = s_pmin[e] = s_smin[e] = edge_len(keys, m, int64_t(L0) - 1 + e);
  __syncthreads();
  for (int off = 1; off < ne; off <<= 1) {  // prefix and suffix minima of the edge lengths
    int a[2], b[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = t + r * kRefitBlock;
      a[r] = e < ne && e >= off ? s_pmin[e - off] : 0x7fffffff;
      b[r] = e + off < ne ? s_smin[e + off] : 0x7fffffff;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = t + r * kRefitBlock;
      if (e < ne) {
        s_pmin[e] = min(s_pmin[e], a[r]);
        s_smin[e] = min(s_smin[e], b[r]);
      }
    }
    __syncthreads();
  }
  const int l = L0 + t;
  if (l >= m) return;
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(node_a, 0, BUF ? m_cap * (16 * kNodeStride) : 0, kBufferWord3);
  auto len = [&](int64_t k) -> int {
    return k >= L0 - 1 && k <= L1 ? s_len[k - (L0 - 1)] : edge_len(keys, m, k);
  };
  Box box = leaf_box<D>(l, xs, n, ls);
  int i = l, j = l;
  int dl = len(i - 1), dr = len(j);
  for (int level = 0; level < m; ++level) {
    if (i == 0 && j == m - 1) return;  // the root, written when it was made
    const bool left = dr > dl;          // this node is its parent's left child
    const int sp = left ? j : i - 1;    // the parent's split
    const bool inside = i >= L0 && j <= L1 &&
                        (left ? sp + 1 <= L1 && s_smin[sp + 1 - (L0 - 1)] < dr
                              : sp >= L0 && s_pmin[sp - 1 - (L0 - 1)] < dl);
    const int mine = left ? i : j;  // this node's far end, seen from the split
    int far;
    Box sib;
    if (inside) {
      const int slot = sp - L0, side = left ? 0 : 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s_side[side][k][slot] = box.lo[k];
        s_side[side][3 + k][slot] = box.hi[k];
      }
      far = __hip_atomic_exchange(&s_far[slot], mine, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (far < 0) return;  // first arriver
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sib.lo[k] = s_side[side ^ 1][k][slot];
        sib.hi[k] = s_side[side ^ 1][3 + k][slot];
      }
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's node stores have landed
      far = atomicExch(ends + sp, mine);
      if (far < 0) return;  // first arriver
      // the sibling: [sp+1, far] (right) or [far, sp] (left); a leaf when it is one key
      const int sl = left ? sp + 1 : sp;
      if (far < 0 || far >= m || (left ? far < sl : far > sl)) {
        atomicOr(info, kInternalBit);
        return;
      }
      if (far == sl) sib = leaf_box<D>(sl, xs, n, ls);
      else sib = BUF ? load_node_buf(rb, sl) : load_node(node_a, node_b, sl);
    }
    const Box own = box;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      box.lo[k] = fminf(box.lo[k], sib.lo[k]);
      box.hi[k] = fmaxf(box.hi[k], sib.hi[k]);
    }
    if (cut) {
      // a child of at most span primitives under a larger parent is a cut node
      const int a0 = left ? i : far, a1 = sp, b0 = sp + 1, b1 = left ? far : j;
      const int span = cut_span(m, cut_div);
      if (b1 - a0 + 1 > span) {
        if (a1 - a0 + 1 <= span)
          cut_add(cut, cut_n, a0 == a1 ? (kLeaf | static_cast<uint32_t>(a1)) : static_cast<uint32_t>(a1), a1,
                  left ? own : sib);
        if (b1 - b0 + 1 <= span)
          cut_add(cut, cut_n, b0 == b1 ? (kLeaf | static_cast<uint32_t>(b0)) : static_cast<uint32_t>(b0), b1,
                  left ? sib : own);
      }
    }
    // the merged node keeps one edge and takes the sibling's far edge
    if (left) {
      j = far;
      dr = len(j);
    } else {
      i = far;
      dl = len(i - 1);
    }
    // the new node's index: its own parent side decides it
    const bool root = i == 0 && j == m - 1;
    const int p = root ? 0 : (dr > dl ? j : i);
    const int o = p == i ? j : i;
    // a record another workgroup reads during this build (its parent's meeting is
    // not in LDS) goes out with agent-scope stores; the others only need to be
    // there for later kernels
    bool shared = false;
    if (!root) {
      const bool l2 = dr > dl;
      const int s2 = l2 ? j : i - 1;
      shared = !(i >= L0 && j <= L1 &&
                 (l2 ? s2 + 1 <= L1 && s_smin[s2 + 1 - (L0 - 1)] < dr : s2 >= L0 && s_pmin[s2 - 1 - (L0 - 1)] < dl));
    }
    if (!shared) {
      node_a[kNodeStride * size_t(p)] = make_float4(box.lo[0], box.lo[1], box.lo[2], __int_as_float(o));
      node_b[kNodeStride * size_t(p)] = make_float4(box.hi[0], box.hi[1], box.hi[2], __int_as_float(sp));
    } else if (BUF) {
      store_node_buf(rb, p, box, o, sp);
    } else {
      store_node(node_a, node_b, p, box, o, sp);
    }
    other[p] = o;
    gamma[p] = sp;
  }
  atomicOr(info, kInternalBit);  // more levels than keys: the keys changed under the build
}

// m_cap: number of primitives, or an upper bound when d_m (device) holds it.
// ends: m_cap words, the far-end exchange of meetings across workgroups.
template <typename K>
void build_t(const K* keys, int m_cap, const int* d_m, int dim, const float* xs, int64_t n_pts,
             const LeafSrc& ls, float4* node_a, float4* node_b, int* rope, int* leaf_rope, int* ends, int* other,
             int* gamma, uint32_t* info, hipStream_t s, float4* cut, int* cut_n, bool ends_ready, int cut_div) {
  if (m_cap <= 0) return;
  int g = static_cast<int>(ceil_div(m_cap, kBlock));
  if (m_cap >= 2) {
    if (!ends_ready) fill_u32(reinterpret_cast<uint32_t*>(ends), 0xffffffffu, m_cap, s);
    const bool buf = m_cap <= kRefitBufMaxNodes;
    const dim3 rg(static_cast<unsigned>(ceil_div(m_cap, kRefitBlock))), rb(kRefitBlock);
    if (dim == 3 && buf)
      hipLaunchKernelGGL((k_build_up<K, 3, true>), rg, rb, 0, s, keys, m_cap, d_m, xs, n_pts, ls, other, gamma, ends,
                         node_a, node_b, info, cut, cut_n, cut_div);
    else if (dim == 3)
      hipLaunchKernelGGL((k_build_up<K, 3, false>), rg, rb, 0, s, keys, m_cap, d_m, xs, n_pts, ls, other, gamma, ends,
                         node_a, node_b, info, cut, cut_n, cut_div);
    else if (buf)
      hipLaunchKernelGGL((k_build_up<K, 2, true>), rg, rb, 0, s, keys, m_cap, d_m, xs, n_pts, ls, other, gamma, ends,
                         node_a, node_b, info, cut, cut_n, cut_div);
    else
      hipLaunchKernelGGL((k_build_up<K, 2, false>), rg, rb, 0, s, keys, m_cap, d_m, xs, n_pts, ls, other, gamma, ends,
                         node_a, node_b, info, cut, cut_n, cut_div);
  }
  hipLaunchKernelGGL(k_ropes, dim3(g), dim3(kBlock), 0, s, other, m_cap, d_m, rope, leaf_rope);
}

}  // namespace

void build_lbvh(const void* keys, bool key64, int m, int dim, const float* xs, int64_t n_pts, const float4* prim_lo,
                const float4* prim_hi, float4* node_a, float4* node_b, int* rope, int* leaf_rope, int* ends,
                int* other, int* gamma, const int* d_m, uint32_t* info, hipStream_t s, float4* cut, int* cut_n,
                bool ends_ready, int cut_div) {
  const LeafSrc ls{prim_lo, prim_hi};
  if (key64)
    build_t(static_cast<const uint64_t*>(keys), m, d_m, dim, xs, n_pts, ls, node_a, node_b, rope, leaf_rope, ends,
            other, gamma, info, s, cut, cut_n, ends_ready, cut_div);
  else
    build_t(static_cast<const uint32_t*>(keys), m, d_m, dim, xs, n_pts, ls, node_a, node_b, rope, leaf_rope, ends,
            other, gamma, info, s, cut, cut_n, ends_ready, cut_div);
}

}  // namespace fdb
