// Traversal kernels: one thread per query point in Morton order (Section 4.1),
// stack-less top-down walks over the LBVH using escape links.
//   core   - preprocessing: count neighbours, stop at minPts (Section 3.2).
//   main   - the fused phase: union (or claim) on discovery, nothing stored
//            (Algorithm 3); the walk is masked so thread i only reaches
//            primitives above its own, handling every pair once (Section 4.1,
//            Figure 1).
//   border - canonical labels: a non-core point takes the smallest cluster id
//            among its core neighbours.
// DenseBox variants (Section 4.2) walk a tree over dense-cell boxes plus the
// points outside dense cells; a box hit scans the cell's points.
#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

struct Query {
  float x, y, z;
};

template <int D>
__device__ __forceinline__ Query load_point(const float* __restrict__ xs, int64_t n, int64_t i) {
  Query q;
  q.x = xs[i];
  q.y = xs[n + i];
  q.z = D == 3 ? xs[2 * n + i] : 0.0f;
  return q;
}

template <int D>
__device__ __forceinline__ bool near(const float* __restrict__ xs, int64_t n, int64_t j, const Query& q, float eps2) {
  float px = xs[j], py = xs[n + j], pz = D == 3 ? xs[2 * n + j] : 0.0f;
  return dist2v<D>(px, py, pz, q.x, q.y, q.z) <= eps2;
}

// Walk the tree, calling visit(prim) for every primitive whose leaf (or bucket)
// the walk reaches; visit returns true to stop. With MASKED, subtrees whose
// primitives all have index <= mask are never entered: at a node whose left
// child ends at or below the mask, the walk goes straight to the right child,
// and buckets start above the mask. Every node the walk reaches then holds a
// primitive above the mask.
//
// A pre-order walk reaches each node at most once, so more than 2m steps, or a
// reference outside the tree, means the tree is broken: the walk then stops and
// raises the internal-error bit instead of looping or reading out of bounds.
template <int D, bool MASKED, typename F>
__device__ __forceinline__ void traverse(const TreeView& t, int m, const Query& q, float eps2, int mask,
                                         uint32_t* info, F&& visit) {
  if (m <= 0) return;
  if (MASKED && mask >= m - 1) return;
  uint32_t node = m == 1 ? kLeaf : 0u;
  int64_t steps = 0;
  const int64_t max_steps = 2 * int64_t(m) + 2;
  while (node != kEnd) {
    if (++steps > max_steps) {
      atomicOr(info, kInternalBit);
      return;
    }
    if (node & kLeaf) {
      int l = static_cast<int>(node & ~kLeaf);
      if (l >= m) {
        atomicOr(info, kInternalBit);
        return;
      }
      if (visit(l)) return;
      node = static_cast<uint32_t>(t.leaf_rope[l]);
      continue;
    }
    if (node >= static_cast<uint32_t>(m - 1)) {
      atomicOr(info, kInternalBit);
      return;
    }
    float4 a = t.node_a[node];
    float4 b = t.node_b[node];
    if (box_dist2<D>(q.x, q.y, q.z, a.x, a.y, a.z, b.x, b.y, b.z) > eps2) {
      node = static_cast<uint32_t>(t.rope[node]);
      continue;
    }
    int k = static_cast<int>(node);
    int o = __float_as_int(a.w), g = __float_as_int(b.w);
    int first = o < k ? o : k, last = o > k ? o : k;
    if (first < 0 || last >= m || g < first || g >= last) {
      atomicOr(info, kInternalBit);
      return;
    }
    if (last - first < t.leaf_size) {
      int s = first;
      if (MASKED && s <= mask) s = mask + 1;
      for (int l = s; l <= last; ++l)
        if (visit(l)) return;
      node = static_cast<uint32_t>(t.rope[node]);
      continue;
    }
    if (MASKED && g <= mask)
      node = last == g + 1 ? (kLeaf | static_cast<uint32_t>(g + 1)) : static_cast<uint32_t>(g + 1);
    else
      node = first == g ? (kLeaf | static_cast<uint32_t>(g)) : static_cast<uint32_t>(g);
  }
}

// True only if `root` is an ancestor of x within a few plain-load hops (then x
// already is in root's set: sets only grow). False means "unknown".
__device__ __forceinline__ bool known_same_set(const int* __restrict__ labels, int x, int root) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    int p = labels[x];
    if (p == root) return true;
    if (p == x) return false;
    x = p;
  }
  return false;
}

__device__ __forceinline__ int tree_m(const TreeView& t) { return t.d_m ? *t.d_m : t.m_cap; }

// ---------------------------------------------------------------- FDbscan ----

template <int D>
__global__ void k_core_fdb(TravArgs a) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= a.n) return;
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  const int need = a.min_pts;
  int cnt = 0;
  traverse<D, false>(a.t, tree_m(a.t), q, eps2, 0, a.info, [&](int j) {
    if (near<D>(a.xs, a.n, j, q, eps2)) return ++cnt >= need;
    return false;
  });
  a.core[i] = cnt >= need ? 1 : 0;
}

template <int D, bool ALL_CORE, bool FIRST>
__global__ void k_main_fdb(TravArgs a) {
  int64_t i64 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i64 >= a.n) return;
  const int i = static_cast<int>(i64);
  const bool ci = ALL_CORE || a.core[i];
  if (!FIRST && !ci) return;  // canonical mode: border points are settled later
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  int* labels = a.labels;
  int root = i;
  traverse<D, true>(a.t, tree_m(a.t), q, eps2, i, a.info, [&](int j) {
    if (!near<D>(a.xs, a.n, j, q, eps2)) return false;
    const bool cj = ALL_CORE || a.core[j];
    if (ci && cj) {
      if (!known_same_set(labels, j, root)) root = uf_union(labels, root, j, a.info);
      return false;
    }
    if (FIRST) {
      if (ci) {
        uf_claim(labels, j, i);
        return false;
      }
      if (cj) {
        uf_claim(labels, i, j);
        return true;  // i is a member now (by this or an earlier claim)
      }
    }
    return false;
  });
}

template <int D>
__global__ void k_border_fdb(TravArgs a) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= a.n) return;
  if (a.core[i]) return;
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  int best = 0x7fffffff;
  traverse<D, false>(a.t, tree_m(a.t), q, eps2, 0, a.info, [&](int j) {
    if (!a.core[j] || !near<D>(a.xs, a.n, j, q, eps2)) return false;
    int c = a.cid[a.labels[j]];
    best = c < best ? c : best;
    return best == 0;
  });
  a.border[i] = best == 0x7fffffff ? -1 : best;
}

// --------------------------------------------------------------- DenseBox ----
// Primitive p covers sorted points [prim_start[p], prim_start[p] + |cnt|):
// cnt > 0 is a single point, cnt < 0 a dense cell (all core, one cluster).

template <int D>
__device__ __forceinline__ bool box_near(const TravArgs& a, int p, const Query& q, float eps2) {
  float4 lo = a.prim_lo[p], hi = a.prim_hi[p];
  return box_dist2<D>(q.x, q.y, q.z, lo.x, lo.y, lo.z, hi.x, hi.y, hi.z) <= eps2;
}

template <int D>
__global__ void k_core_dbx(TravArgs a) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= a.n) return;
  if (a.core[i]) return;  // points of dense cells are core by construction
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  const int need = a.min_pts;
  int cnt = 0;
  traverse<D, false>(a.t, tree_m(a.t), q, eps2, 0, a.info, [&](int p) {
    int c = a.prim_cnt[p], s = a.prim_start[p];
    if (c > 0) {
      if (near<D>(a.xs, a.n, s, q, eps2)) return ++cnt >= need;
      return false;
    }
    if (!box_near<D>(a, p, q, eps2)) return false;
    for (int j = s; j < s - c; ++j)
      if (near<D>(a.xs, a.n, j, q, eps2) && ++cnt >= need) return true;
    return false;
  });
  a.core[i] = cnt >= need ? 1 : 0;
}

template <int D, bool ALL_CORE, bool FIRST>
__global__ void k_main_dbx(TravArgs a) {
  int64_t i64 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i64 >= a.n) return;
  const int i = static_cast<int>(i64);
  const bool ci = ALL_CORE || a.core[i];
  if (!FIRST && !ci) return;
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  int* labels = a.labels;
  int root = labels[i];  // a dense cell's points start out pointing at its first point
  const int own = a.prim_of[i];
  traverse<D, true>(a.t, tree_m(a.t), q, eps2, own, a.info, [&](int p) {
    int c = a.prim_cnt[p], s = a.prim_start[p];
    if (c > 0) {
      const int j = s;
      if (!near<D>(a.xs, a.n, j, q, eps2)) return false;
      const bool cj = ALL_CORE || a.core[j];
      if (ci && cj) {
        if (!known_same_set(labels, j, root)) root = uf_union(labels, root, j, a.info);
        return false;
      }
      if (FIRST) {
        if (ci) {
          uf_claim(labels, j, i);
          return false;
        }
        if (cj) {
          uf_claim(labels, i, j);
          return true;
        }
      }
      return false;
    }
    // a dense cell: one point within eps suffices (its points are all core and
    // already share one set)
    if (!box_near<D>(a, p, q, eps2)) return false;
    if (ci && known_same_set(labels, s, root)) return false;
    for (int j = s; j < s - c; ++j) {
      if (!near<D>(a.xs, a.n, j, q, eps2)) continue;
      if (ci) {
        root = uf_union(labels, root, s, a.info);
        return false;
      }
      if (FIRST) {
        uf_claim(labels, i, s);
        return true;
      }
      return false;
    }
    return false;
  });
}

template <int D>
__global__ void k_border_dbx(TravArgs a) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= a.n) return;
  if (a.core[i]) return;
  const Query q = load_point<D>(a.xs, a.n, i);
  const float eps2 = a.eps2;
  int best = 0x7fffffff;
  traverse<D, false>(a.t, tree_m(a.t), q, eps2, 0, a.info, [&](int p) {
    int c = a.prim_cnt[p], s = a.prim_start[p];
    if (c > 0) {
      if (!a.core[s] || !near<D>(a.xs, a.n, s, q, eps2)) return false;
      int id = a.cid[a.labels[s]];
      best = id < best ? id : best;
      return best == 0;
    }
    if (!box_near<D>(a, p, q, eps2)) return false;
    int id = a.cid[a.labels[s]];
    if (id >= best) return false;
    for (int j = s; j < s - c; ++j) {
      if (near<D>(a.xs, a.n, j, q, eps2)) {
        best = id;
        return best == 0;
      }
    }
    return false;
  });
  a.border[i] = best == 0x7fffffff ? -1 : best;
}

inline dim3 grid_of(int64_t n, int block) { return dim3(static_cast<unsigned>(ceil_div(n, block))); }

}  // namespace

void launch_core(const TravArgs& a, int dim, bool densebox, hipStream_t s) {
  if (a.n <= 0) return;
  dim3 g = grid_of(a.n, a.block), b(a.block);
  if (densebox) {
    if (dim == 3) hipLaunchKernelGGL(k_core_dbx<3>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_core_dbx<2>, g, b, 0, s, a);
  } else {
    if (dim == 3) hipLaunchKernelGGL(k_core_fdb<3>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_core_fdb<2>, g, b, 0, s, a);
  }
}

template <int D, bool ALL, bool FIRST>
static void main_t(const TravArgs& a, bool densebox, hipStream_t s) {
  dim3 g = grid_of(a.n, a.block), b(a.block);
  if (densebox) hipLaunchKernelGGL((k_main_dbx<D, ALL, FIRST>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_main_fdb<D, ALL, FIRST>), g, b, 0, s, a);
}

void launch_main(const TravArgs& a, int dim, bool densebox, bool all_core, bool first_border, hipStream_t s) {
  if (a.n <= 0) return;
  if (dim == 3) {
    if (all_core) main_t<3, true, false>(a, densebox, s);
    else if (first_border) main_t<3, false, true>(a, densebox, s);
    else main_t<3, false, false>(a, densebox, s);
  } else {
    if (all_core) main_t<2, true, false>(a, densebox, s);
    else if (first_border) main_t<2, false, true>(a, densebox, s);
    else main_t<2, false, false>(a, densebox, s);
  }
}

void launch_border(const TravArgs& a, int dim, bool densebox, hipStream_t s) {
  if (a.n <= 0) return;
  dim3 g = grid_of(a.n, a.block), b(a.block);
  if (densebox) {
    if (dim == 3) hipLaunchKernelGGL(k_border_dbx<3>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_border_dbx<2>, g, b, 0, s, a);
  } else {
    if (dim == 3) hipLaunchKernelGGL(k_border_fdb<3>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_border_fdb<2>, g, b, 0, s, a);
  }
}

}  // namespace fdb
