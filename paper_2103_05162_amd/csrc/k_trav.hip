// Traversal kernels: one query per lane in Morton order (Section 4.1),
// stack-less top-down walks over the LBVH using escape links.
//   core   - preprocessing: count neighbours, stop at minPts (Section 3.2).
//   main   - the fused phase: union (or claim) on discovery, nothing stored
//            (Algorithm 3); the walk is masked so query i only reaches
//            primitives above its own, handling every pair once (Section 4.1,
//            Figure 1).
//   border - canonical labels: a non-core point takes the smallest cluster id
//            among its core neighbours.
// DenseBox variants (Section 4.2) walk a tree over dense-cell boxes plus the
// points outside dense cells; a box hit scans the cell's points.
//
// Every walk has a scope: the subtree it starts from, the last primitive of
// that subtree, eps^2 and minPts. A single cloud's scope is the whole tree; in
// a batch the keys carry the cloud id above the Morton bits, so each cloud is
// one subtree, and a query's scope is its cloud's (with its own eps, minPts).
#include <algorithm>

#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

struct Query {
  float x, y, z;
};

struct Scope {
  uint32_t start;  // first node of the walk (internal node, or kLeaf | leaf)
  int end;         // last primitive of the subtree
  float eps2;
  int min_pts;
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

__device__ __forceinline__ int tree_m(const TreeView& t) { return t.d_m ? *t.d_m : t.m_cap; }

__device__ __forceinline__ int cloud_of(const TravArgs& a, int i) {
  return min(static_cast<int>(a.pkeys[i] >> a.key_shift), a.num_clouds - 1);
}

// Scope of the query at sorted point index i.
template <bool BATCHED>
__device__ __forceinline__ Scope scope_of(const TravArgs& a, int m, int i) {
  Scope s;
  if (BATCHED) {
    const int c = cloud_of(a, i);
    s.start = static_cast<uint32_t>(a.cloud_root[c]);
    s.end = a.cloud_end[c];
    s.eps2 = a.cloud_eps2[c];
    s.min_pts = a.cloud_minpts[c];
  } else {
    s.start = m == 1 ? kLeaf : 0u;
    s.end = m - 1;
    s.eps2 = a.eps2;
    s.min_pts = a.min_pts;
  }
  return s;
}

// Walk the subtree of sc, calling visit(prim) for every primitive whose leaf
// (or bucket) the walk reaches; visit returns true to stop. With MASKED,
// subtrees whose primitives all have index <= mask are never entered: at a node
// whose left child ends at or below the mask, the walk goes straight to the
// right child, and buckets start above the mask. Every node the walk reaches
// then holds a primitive above the mask. The walk ends where an escape link
// would leave the subtree (past primitive sc.end).
//
// A pre-order walk reaches each node at most once, so more than 2m steps, or a
// reference outside the tree, means the tree is broken: the walk then stops and
// raises the internal-error bit instead of looping or reading out of bounds.
template <int D, bool MASKED, typename F>
__device__ __forceinline__ void traverse(const TreeView& t, int m, const Scope& sc, const Query& q, int mask,
                                         uint32_t* info, F&& visit) {
  if (m <= 0) return;
  if (MASKED && mask >= sc.end) return;
  uint32_t node = sc.start;
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
      if (visit(l) || l >= sc.end) return;
      node = static_cast<uint32_t>(t.leaf_rope[l]);
      continue;
    }
    if (node >= static_cast<uint32_t>(m - 1)) {
      atomicOr(info, kInternalBit);
      return;
    }
    // the escape link is loaded with the node, not after its box test fails
    const float4 a = t.node_a[kNodeStride * size_t(node)];
    const float4 b = t.node_b[kNodeStride * size_t(node)];
    const uint32_t esc = static_cast<uint32_t>(t.rope[node]);
    const int k = static_cast<int>(node);
    const int o = __float_as_int(a.w), g = __float_as_int(b.w);
    const int first = o < k ? o : k, last = o > k ? o : k;
    if (box_dist2<D>(q.x, q.y, q.z, a.x, a.y, a.z, b.x, b.y, b.z) > sc.eps2) {
      if (last >= sc.end) return;
      node = esc;
      continue;
    }
    if (first < 0 || last >= m || g < first || g >= last) {
      atomicOr(info, kInternalBit);
      return;
    }
    if (last - first < t.leaf_size) {
      int s = first;
      if (MASKED && s <= mask) s = mask + 1;
      for (int l = s; l <= last; ++l)
        if (visit(l)) return;
      if (last >= sc.end) return;
      node = esc;
      continue;
    }
    if (MASKED && g <= mask)
      node = last == g + 1 ? (kLeaf | static_cast<uint32_t>(g + 1)) : static_cast<uint32_t>(g + 1);
    else
      node = first == g ? (kLeaf | static_cast<uint32_t>(g)) : static_cast<uint32_t>(g);
  }
}

// Wave-uniform walk for a box query (every point of box [lo,hi]), masked like
// traverse(): visit(first, last) is called with the same primitive range on
// every lane, for each bucket (a subtree of at most leaf_size primitives, cut
// to primitives above the mask) and each single leaf the walk reaches.
template <int D, typename F>
__device__ __forceinline__ bool traverse_box(const TreeView& t, int m, const Scope& sc, const float* lo,
                                             const float* hi, int mask, int leaf_size, uint32_t* info, F&& visit) {
  if (m <= 0 || mask >= sc.end) return false;
  uint32_t node = sc.start;
  int64_t steps = 0;
  const int64_t max_steps = 2 * int64_t(m) + 2;
  while (node != kEnd) {
    node = __builtin_amdgcn_readfirstlane(node);
    if (++steps > max_steps) {
      atomicOr(info, kInternalBit);
      return false;
    }
    if (node & kLeaf) {
      int l = static_cast<int>(node & ~kLeaf);
      if (l >= m) {
        atomicOr(info, kInternalBit);
        return false;
      }
      if (visit(l, l)) return true;
      if (l >= sc.end) return false;
      node = static_cast<uint32_t>(t.leaf_rope[l]);
      continue;
    }
    if (node >= static_cast<uint32_t>(m - 1)) {
      atomicOr(info, kInternalBit);
      return false;
    }
    const float4 na = t.node_a[kNodeStride * size_t(node)];
    const float4 nb = t.node_b[kNodeStride * size_t(node)];
    const uint32_t esc = static_cast<uint32_t>(t.rope[node]);
    const int k = static_cast<int>(node);
    const int o = __float_as_int(na.w), g = __float_as_int(nb.w);
    const int first = o < k ? o : k, last = o > k ? o : k;
    if (boxbox_dist2<D>(lo, hi, na.x, na.y, na.z, nb.x, nb.y, nb.z) > sc.eps2) {
      if (last >= sc.end) return false;
      node = esc;
      continue;
    }
    if (first < 0 || last >= m || g < first || g >= last) {
      atomicOr(info, kInternalBit);
      return false;
    }
    if (last - first < leaf_size) {
      int s = first <= mask ? mask + 1 : first;
      if (s <= last && visit(s, last)) return true;
      if (last >= sc.end) return false;
      node = esc;
      continue;
    }
    if (g <= mask)
      node = last == g + 1 ? (kLeaf | static_cast<uint32_t>(g + 1)) : static_cast<uint32_t>(g + 1);
    else
      node = first == g ? (kLeaf | static_cast<uint32_t>(g)) : static_cast<uint32_t>(g);
  }
  return false;
}

// Wavefront-cooperative form of traverse_box: the wavefront expands up to 64
// tree nodes per step (one per lane) from its own stack in LDS, newest first,
// so a walk takes about as many steps as the tree is deep instead of one step
// per node. Every bucket and leaf that one step reaches is handed out a
// primitive per lane, visit_lanes(r) being called on the whole wavefront with
// each lane's own primitive (-1 for none), so the visitor loads all of them at
// once. It visits the same buckets and leaves as traverse_box (in another order:
// callers only union, which does not depend on it). Children that do not fit on
// the stack have their subtrees walked with traverse_box instead. SKIP: cut
// subtrees that t.cut_sum marks as holding no core point, or as already in the
// set of root skip_root (labels skip_labels), are not walked.
constexpr int kWideStack = 512;  // entries per wavefront

template <int D, bool SKIP = false, typename F>
__device__ __forceinline__ void traverse_box_wide_lanes(const TreeView& t, int m, const Scope& sc, const float* lo,
                                                        const float* hi, int mask, int leaf_size, uint32_t* info,
                                                        uint32_t* stack, F&& visit_lanes,
                                                        const int* skip_labels = nullptr, int skip_root = -1) {
  if (m <= 0 || mask >= sc.end) return;
  const int lane = lane_id();
  // a range [s, e] of one lane (wave-uniform arguments), 64 primitives per call
  auto range = [&](int s, int e) {
    for (int b = s; b <= e; b += 64)
      if (visit_lanes(b + lane <= e ? b + lane : -1)) return true;
    return false;
  };
  int top = 0;
  // a walk over the whole tree starts from the cut: its boxes are tested 64 at a
  // time and the ones within reach pushed, instead of descending from the root
  const int nc = t.cut && sc.start == 0 && sc.end == m - 1 ? *t.cut_n : 0;
  if (nc > 0 && nc <= kCutMax) {
    for (int b = 0; b < nc && top >= 0; b += 64 * kCutUnroll) {
      float4 ca[kCutUnroll], cb[kCutUnroll];
      int cs[kCutUnroll];
#pragma unroll
      for (int u = 0; u < kCutUnroll; ++u) {  // the loads of kCutUnroll chunks in flight together
        const int c = min(b + u * 64 + lane, nc - 1);
        ca[u] = t.cut[2 * c];
        cb[u] = t.cut[2 * c + 1];
        cs[u] = SKIP && t.cut_sum ? t.cut_sum[c] : kCutMixed;
      }
#pragma unroll
      for (int u = 0; u < kCutUnroll; ++u) {
        bool hit = b + u * 64 + lane < nc && __float_as_int(cb[u].w) > mask &&
                   boxbox_dist2<D>(lo, hi, ca[u].x, ca[u].y, ca[u].z, cb[u].x, cb[u].y, cb[u].z) <= sc.eps2;
        // a subtree without core points, or one whose core points were all in the
        // walker's set (skip_root) when summarised, adds no union: sets only merge
        if (SKIP && hit && cs[u] != kCutMixed)
          hit = !(cs[u] == kCutNoCore ||
                  (skip_root >= 0 && (cs[u] == skip_root || skip_labels[cs[u]] == skip_root)));
        const uint64_t hm = ballot(hit);
        if (top < 0 || top + __popcll(hm) > kWideStack) {
          top = -1;  // more than the stack holds: start from the root instead
        } else {
          if (hit) stack[top + __popcll(hm & lanemask_lt())] = __float_as_uint(ca[u].w);
          top += __popcll(hm);
        }
      }
    }
  }
  if (nc <= 0 || nc > kCutMax || top < 0) {
    if (lane == 0) stack[0] = sc.start;
    top = 1;
  }
  int64_t guard = 0;
  const int64_t max_rounds = 2 * int64_t(m) + 2;
  while (top > 0) {
    if (++guard > max_rounds) {
      atomicOr(info, kInternalBit);
      return;
    }
    const int take = top < 64 ? top : 64;
    top -= take;
    const uint32_t node = lane < take ? stack[top + lane] : kEnd;
    int bs = -1, be = -1;
    uint32_t c0 = kEnd, c1 = kEnd;
    if (node != kEnd) {
      if (node & kLeaf) {
        const int l = static_cast<int>(node & ~kLeaf);
        if (l >= m) atomicOr(info, kInternalBit);
        else if (l > mask) bs = be = l;
      } else if (node >= static_cast<uint32_t>(m - 1)) {
        atomicOr(info, kInternalBit);
      } else {
        const float4 na = t.node_a[kNodeStride * size_t(node)];
        const float4 nb = t.node_b[kNodeStride * size_t(node)];
        const int k = static_cast<int>(node);
        const int o = __float_as_int(na.w), g = __float_as_int(nb.w);
        const int first = o < k ? o : k, last = o > k ? o : k;
        if (last > mask && boxbox_dist2<D>(lo, hi, na.x, na.y, na.z, nb.x, nb.y, nb.z) <= sc.eps2) {
          if (first < 0 || last >= m || g < first || g >= last) {
            atomicOr(info, kInternalBit);
          } else if (last - first < leaf_size) {
            bs = first <= mask ? mask + 1 : first;
            be = last;
          } else {
            if (g > mask) c0 = first == g ? (kLeaf | static_cast<uint32_t>(g)) : static_cast<uint32_t>(g);
            c1 = last == g + 1 ? (kLeaf | static_cast<uint32_t>(g + 1)) : static_cast<uint32_t>(g + 1);
          }
        }
      }
    }
    // this step's buckets laid end to end over the lanes: slot k of round q is
    // primitive q*64 + lane of the concatenation, found by a binary search over the
    // lanes' exclusive prefix sums (the last lane starting at or before it)
    const int len = bs >= 0 ? be - bs + 1 : 0;
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    const int excl = incl - len;
    const int total = __shfl(incl, 63);
    for (int q = 0; q < total; q += 64) {  // every lane takes part in the shuffles
      const int slot = q + lane;
      const int sl = slot < total ? slot : total - 1;
      int lo = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (__shfl(excl, lo + step) <= sl) lo += step;
      const int first = __shfl(bs, lo), ex = __shfl(excl, lo);
      if (visit_lanes(slot < total ? first + (sl - ex) : -1)) return;
    }
    const uint64_t m0 = ballot(c0 != kEnd), m1 = ballot(c1 != kEnd);
    const int n0 = __popcll(m0), n1 = __popcll(m1);
    if (top + n0 + n1 <= kWideStack) {
      const uint64_t lt = lanemask_lt();
      if (c0 != kEnd) stack[top + __popcll(m0 & lt)] = c0;
      if (c1 != kEnd) stack[top + n0 + __popcll(m1 & lt)] = c1;
      top += n0 + n1;
    } else {
      // stack full: walk each child's subtree on its own
      for (uint64_t cm = m0 | m1; cm; cm &= cm - 1) {
        const int L = __ffsll(static_cast<unsigned long long>(cm)) - 1;
        for (int side = 0; side < 2; ++side) {
          const uint32_t c = static_cast<uint32_t>(__shfl(static_cast<int>(side ? c1 : c0), L));
          if (c == kEnd) continue;
          int end;
          if (c & kLeaf) {
            end = static_cast<int>(c & ~kLeaf);
          } else {
            const int oc = __float_as_int(t.node_a[kNodeStride * size_t(c)].w);
            end = oc > static_cast<int>(c) ? oc : static_cast<int>(c);
          }
          const Scope sub{c, end, sc.eps2, sc.min_pts};
          if (traverse_box<D>(t, m, sub, lo, hi, mask, leaf_size, info, range)) return;
        }
      }
    }
  }
}

// True only if `root` is an ancestor of x within a few plain-load hops (then x
// already is in root's set: sets only grow). False means "unknown". When the
// chain had intermediate links, x is re-pointed straight at root (an ancestor,
// so the store is safe however it races) and the next check is one load.
__device__ __forceinline__ bool known_same_set(int* labels, int x, int root) {
  const int x0 = x;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    int p = labels[x];
    if (p == root) {
      if (h > 0) labels[x0] = root;
      return true;
    }
    if (p == x) return false;
    x = p;
  }
  return false;
}

// Slot in a list (counter *n) for every thread where pred holds, -1 elsewhere:
// one atomic per workgroup, threads in order within it. Every thread of the
// workgroup must call it (it synchronises the workgroup); s_w holds 17 ints.
__device__ __forceinline__ int block_reserve(int* n, bool pred, int* s_w) {
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
  const int slot = s_w[16] + s_w[w] + __popcll(b & lanemask_lt());
  __syncthreads();
  return pred ? slot : -1;
}

// Up to kRecNb neighbouring primitives of one query, kept in LDS: row t of the
// workgroup's table (kRecNb x blockDim ints, dynamic shared memory) holds every
// thread's t-th neighbour, so a neighbour costs one store.
struct NbRec {
  int* col;  // &table[0][threadIdx.x]; entry t at col[t * blockDim.x]
  int nn;
};

__device__ __forceinline__ void rec_init(NbRec& r, int* table) {
  r.col = table + threadIdx.x;
  r.nn = 0;
}

__device__ __forceinline__ void rec_add(NbRec& r, int j) {
  if (r.nn < kRecNb) r.col[r.nn * blockDim.x] = j;
  ++r.nn;
}

__device__ __forceinline__ int rec_get(const NbRec& r, int t) { return r.col[t * blockDim.x]; }

// Records tell a dense cell (stored as -2 - its first point) from a point.
__device__ __forceinline__ int cell_ref(int s) { return -2 - s; }
__device__ __forceinline__ bool is_cell_ref(int v) { return v < -1; }
__device__ __forceinline__ int ref_point(int v) { return v < -1 ? -2 - v : v; }

// End of a core pass for query point i (primitive p): core and lone flags, and
// what the border pass will need: nothing (core, or lone: border -1 now), a
// neighbour record, or a walk. Called by every thread of the workgroup.
__device__ __forceinline__ void core_epilogue(const TravArgs& a, bool mine, int i, int p, int cnt, int min_pts,
                                              const NbRec& rec, int* s_w) {
  const bool core = mine && cnt >= min_pts;
  const bool lone = mine && cnt <= 1 && !core;
  if (mine) {
    a.core[i] = core ? 1 : 0;
    a.lone[i] = lone ? 1 : 0;
    if (lone) a.border[i] = -1;
  }
  if (core) {
    // A core point and a dense cell it reaches are a core pair: join them now,
    // so the main phase finds them in one set and skips the cell scan.
    const int nr = rec.nn < kRecNb ? rec.nn : kRecNb;
    int root = i;
    for (int t = 0; t < nr; ++t) {
      const int v = rec_get(rec, t);
      if (is_cell_ref(v)) root = uf_union(a.labels, root, ref_point(v), a.info);
    }
  }
  const bool want = mine && !core && !lone;
  const bool fits = want && rec.nn <= kRecNb;
  const int slot = block_reserve(a.brec_n, fits, s_w);
  const bool stored = fits && slot < a.brec_cap;
  if (stored) {
    a.brec_i[slot] = i;
#pragma unroll
    for (int t = 0; t < kRecNb; ++t)
      a.brec_nb[int64_t(slot) * kRecNb + t] = t < rec.nn ? ref_point(rec_get(rec, t)) : -1;
  }
  const int wslot = block_reserve(a.qborder_n, want && !stored, s_w);
  if (wslot >= 0) a.qborder[wslot] = p;
}

// A non-core point with no neighbour but itself (known once the core pass has
// run) is noise: nothing to claim, no cluster to join.
__device__ __forceinline__ bool is_lone(const TravArgs& a, int i) { return a.lone && a.lone[i]; }

// An ancestor of x close to its root: labels followed for up to 16 hops, all
// lanes of a bucket at once. Equal to a query's root means the two are already
// in one set (sets only grow); anything else only means "unknown". When the chain
// had more than one link, x is re-pointed straight at the ancestor found (an
// ancestor stays an ancestor, so the store is safe however it races): points are
// visited by many walks, and the next visit takes one load (FDbscan main phase on
// the 8M set 37.4 -> 35.2 ms).
__device__ __forceinline__ int ancestor_compress(int* labels, int x) {
  const int x0 = x;
  int p = labels[x];
  int h = 0;
#pragma unroll 1
  for (; h < 16 && p != x; ++h) {
    x = p;
    p = labels[x];
  }
  if (h > 1) labels[x0] = p;
  return p;
}

__device__ __forceinline__ float readlane_f(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// ---------------------------------------------------------------- FDbscan ----

template <int D, bool B>
__global__ void k_core_fdb(TravArgs a) {
  __shared__ int s_w[17];
  extern __shared__ int s_rec[];  // kRecNb * blockDim.x
  const int64_t i64 = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, a.n);
  const bool mine = i64 >= 0 && i64 < a.n;
  const int i = mine ? static_cast<int>(i64) : 0;
  const int m = tree_m(a.t);
  const Scope sc = scope_of<B>(a, m, i);
  const Query q = load_point<D>(a.xs, a.n, i);
  int cnt = 0;
  NbRec rec;
  rec_init(rec, s_rec);
  if (mine)
    traverse<D, false>(a.t, m, sc, q, 0, a.info, [&](int j) {
      if (!near<D>(a.xs, a.n, j, q, sc.eps2)) return false;
      if (j != i) rec_add(rec, j);
      return ++cnt >= sc.min_pts;
    });
  core_epilogue(a, mine, i, i, cnt, sc.min_pts, rec, s_w);
}

// First-claim main phase (the paper's border rule): per-lane walks, or a packet
// walk when the wavefront's queries lie in a small box. In a packet each lane
// still decides its own pairs.
__device__ __forceinline__ void main_pair_first(const TravArgs& a, int i, bool ci, int j, bool cj, int& root,
                                                bool& done) {
  int* labels = a.labels;
  if (ci && cj) {
    if (!known_same_set(labels, j, root)) root = uf_union(labels, root, j, a.info);
  } else if (ci) {
    uf_claim(labels, j, i);
  } else if (cj) {
    uf_claim(labels, i, j);
    done = true;  // i is a member now (by this or an earlier claim)
  }
}

template <int D, bool B>
__global__ void k_main_fdb_first(TravArgs a) {
  const int64_t i64 = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, a.n);
  const bool valid = i64 >= 0 && i64 < a.n;
  const int i = valid ? static_cast<int>(i64) : 0;
  const bool ci = valid && a.core[i];
  const bool mine = valid && (ci || !is_lone(a, i));
  const int m = tree_m(a.t);
  const Scope sc = scope_of<B>(a, m, i);
  const Query q = load_point<D>(a.xs, a.n, i);
  int root = i;
  bool done = !mine;
  const uint64_t any_mine = ballot(mine);
  if (!any_mine) return;
  const int first_lane = __ffsll(static_cast<unsigned long long>(any_mine)) - 1;
  float lo[3], hi[3];
  lo[0] = mine ? q.x : INFINITY; hi[0] = mine ? q.x : -INFINITY;
  lo[1] = mine ? q.y : INFINITY; hi[1] = mine ? q.y : -INFINITY;
  lo[2] = mine ? q.z : INFINITY; hi[2] = mine ? q.z : -INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
    }
  float ext = fmaxf(hi[0] - lo[0], hi[1] - lo[1]);
  if (D == 3) ext = fmaxf(ext, hi[2] - lo[2]);
  const int c0 = B ? __shfl(cloud_of(a, i), first_lane) : 0;
  const bool one_cloud = !B || !ballot(mine && cloud_of(a, i) != c0);
  const int i0 = __shfl(i, first_lane);
  const Scope ps = scope_of<B>(a, m, i0);
  if (one_cloud && ext * ext <= a.packet_ext_eps2 * ps.eps2) {
    const int lane = lane_id();
    traverse_box<D>(a.t, m, ps, lo, hi, i0, a.packet_leaf, a.info, [&](int s, int e) {
      const int cnt = e - s + 1;  // <= packet_leaf <= 64
      float cx = 0.0f, cy = 0.0f, cz = 0.0f;
      int cc = 0;
      if (lane < cnt) {
        const int j = s + lane;
        cx = a.xs[j];
        cy = a.xs[a.n + j];
        cz = D == 3 ? a.xs[2 * a.n + j] : 0.0f;
        cc = a.core[j] ? 1 : 0;
      }
      for (int k = 0; k < cnt; ++k) {
        const int j = s + k;
        const bool cj = __builtin_amdgcn_readlane(cc, k) != 0;
        const bool act = !done && j > i;
        if (!ballot(act)) continue;
        const float px = readlane_f(cx, k), py = readlane_f(cy, k), pz = readlane_f(cz, k);
        if (act && dist2v<D>(px, py, pz, q.x, q.y, q.z) <= ps.eps2) main_pair_first(a, i, ci, j, cj, root, done);
      }
      return false;
    });
    return;
  }
  if (!mine) return;
  traverse<D, true>(a.t, m, sc, q, i, a.info, [&](int j) {
    if (!near<D>(a.xs, a.n, j, q, sc.eps2)) return false;
    main_pair_first(a, i, ci, j, a.core[j] != 0, root, done);
    return done;
  });
}

// Before FDbscan's packet main phase: each core point joins the core points among
// the next kLocalWindow along the curve that are within eps (pairs of the main
// phase, taken early: in a dense clump consecutive points are close, so a clump
// ends up in one or a few sets), so that the cut summaries below find whole
// subtrees already in one set.
constexpr int kLocalWindow = 8;

template <int D, bool ALL_CORE>
__global__ __launch_bounds__(256) void k_fdb_local(TravArgs a) {
  const int64_t i64 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i64 >= a.n) return;
  const int i = static_cast<int>(i64);
  if (!(ALL_CORE || a.core[i])) return;
  const Query q = load_point<D>(a.xs, a.n, i);
  int root = i;
  for (int u = 1; u <= kLocalWindow; ++u) {
    const int j = i + u;
    if (j >= a.n) break;
    if (!(ALL_CORE || a.core[j]) || !near<D>(a.xs, a.n, j, q, a.eps2)) continue;
    if (!known_same_set(a.labels, j, root)) root = uf_union(a.labels, root, j, a.info);
  }
}

// Summary of cut subtree c (a workgroup each): the root of every core point under
// it (kCutNoCore: none; kCutMixed: more than one, or a chain too long to follow).
template <bool ALL_CORE>
__global__ __launch_bounds__(256) void k_cut_summary(TreeView t, int m, const int* __restrict__ labels,
                                                     const uint8_t* __restrict__ core, int* __restrict__ sum) {
  __shared__ int s_lo[4], s_hi[4];
  const int nc = *t.cut_n;
  const int c = blockIdx.x;
  if (nc > kCutMax || c >= nc) return;  // whole workgroup
  const float4 ca = t.cut[2 * c], cb = t.cut[2 * c + 1];
  const uint32_t ref = __float_as_uint(ca.w);
  const int last = __float_as_int(cb.w);
  int first = last;
  if (!(ref & kLeaf) && ref < static_cast<uint32_t>(m - 1)) {
    const int k = static_cast<int>(ref);
    const int o = __float_as_int(t.node_a[kNodeStride * size_t(k)].w);
    first = o < k ? o : k;
  }
  int lo = 0x7fffffff, hi = -1;  // smallest and largest root among the core points
  if (first < 0 || last >= m || first > last) lo = -3;  // not a range: never skipped
  for (int i = first + static_cast<int>(threadIdx.x); lo != -3 && i <= last; i += 256) {
    if (!(ALL_CORE || core[i])) continue;
    int x = i, p = labels[x];
    for (int h = 0; p != x && h < 64; ++h) {
      x = p;
      p = labels[x];
    }
    if (p != x) {
      lo = -3;  // mixed
      break;
    }
    lo = x < lo ? x : lo;
    hi = x > hi ? x : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off));
    hi = max(hi, __shfl_xor(hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    s_lo[threadIdx.x >> 6] = lo;
    s_hi[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    sum[c] = lo == -3 ? kCutMixed : (hi < 0 ? kCutNoCore : (lo == hi ? lo : kCutMixed));
  }
}

// Canonical (and minPts <= 2) main phase, Q queries per lane: a wavefront owns
// 64*Q consecutive queries. When they lie in a small box (and, in a batch, in
// one cloud) they walk as one packet: the lanes load a bucket of candidates
// once and broadcast it. Phase A unions the packet's own pairs; if then every
// query shares one root r, a candidate whose label is r is skipped untested and
// a candidate within eps of any query costs one union for the whole packet.
template <int D, bool ALL_CORE, bool B, int Q>
__global__ __launch_bounds__(256) void k_main_fdb_q(TravArgs a) {
  __shared__ uint32_t s_stack[4 * kWideStack];  // packet walks (256-thread workgroups)
  const int lane = lane_id();
  const int64_t bbase = xcd_spread(blockIdx.x, 256 * Q, 0, a.n);
  if (bbase < 0) return;
  const int64_t base = bbase + int64_t(threadIdx.x >> 6) * 64 * Q;  // this wavefront's first query
  if (base >= a.n) return;
  const int m = tree_m(a.t);
  int* labels = a.labels;
  int idx[Q], root[Q];
  bool mine[Q];
  Query q[Q];
  uint64_t mm[Q];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const int64_t i64 = base + s * 64 + lane;
    const bool valid = i64 < a.n;
    idx[s] = valid ? static_cast<int>(i64) : 0;
    mine[s] = valid && (ALL_CORE || a.core[idx[s]]);
    q[s] = load_point<D>(a.xs, a.n, idx[s]);
    root[s] = idx[s];
    if (mine[s]) {
      lo[0] = fminf(lo[0], q[s].x); hi[0] = fmaxf(hi[0], q[s].x);
      lo[1] = fminf(lo[1], q[s].y); hi[1] = fmaxf(hi[1], q[s].y);
      lo[2] = fminf(lo[2], q[s].z); hi[2] = fmaxf(hi[2], q[s].z);
    }
    mm[s] = ballot(mine[s]);
  }
  uint64_t any = 0;
#pragma unroll
  for (int s = 0; s < Q; ++s) any |= mm[s];
  if (!any) return;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
    }
  float ext = fmaxf(hi[0] - lo[0], hi[1] - lo[1]);
  if (D == 3) ext = fmaxf(ext, hi[2] - lo[2]);
  int first_slot = 0;
#pragma unroll
  for (int s = Q - 1; s >= 0; --s)
    if (mm[s]) first_slot = s;
  const int fl = __ffsll(static_cast<unsigned long long>(mm[first_slot])) - 1;
  const int i0 = static_cast<int>(base) + first_slot * 64 + fl;
  const Scope ps = scope_of<B>(a, m, i0);
  bool other_cloud = false;
  if (B) {
#pragma unroll
    for (int s = 0; s < Q; ++s) other_cloud |= mine[s] && cloud_of(a, idx[s]) != cloud_of(a, i0);
  }
  const bool packet = !ballot(other_cloud) && ext * ext <= a.packet_ext_eps2 * ps.eps2;

  if (!ALL_CORE && !packet && a.t.cut_sum && !B) {
    // spread out, with cut summaries and minPts > 2 (so every query is a core
    // point, in a dense neighbourhood): each query walks as a packet of one (the
    // lane-wide walk, passing over cut subtrees already in its set). Per-lane
    // rope walks of a wavefront of such queries at a clump's edge took 13-15 ms,
    // each lane visiting the clump's candidates one by one. With minPts <= 2
    // every point is a query and sparse ones walk cheaply on their own lanes
    // (a 2M-point friends-of-friends set: 5.0 ms that way, 11.1 ms as packets of one).
    uint32_t* qstack = s_stack + (threadIdx.x >> 6) * kWideStack;
#pragma unroll
    for (int s = 0; s < Q; ++s)
      for (uint64_t qm = mm[s]; qm; qm &= qm - 1) {
        const int kl = __ffsll(static_cast<unsigned long long>(qm)) - 1;
        const int i = __builtin_amdgcn_readlane(idx[s], kl);
        const float qx = readlane_f(q[s].x, kl), qy = readlane_f(q[s].y, kl), qz = readlane_f(q[s].z, kl);
        const float qb[3] = {qx, qy, qz};
        const Scope sc = scope_of<B>(a, m, i);
        int r = 0;
        if (lane == 0) r = uf_find(labels, i, a.info);
        r = __shfl(r, 0);
        traverse_box_wide_lanes<D, true>(a.t, m, sc, qb, qb, i, a.packet_leaf, a.info, qstack, [&](int jl) {
          bool hit = false;
          if (jl > i && (ALL_CORE || a.core[jl]))
            hit = dist2v<D>(a.xs[jl], a.xs[a.n + jl], D == 3 ? a.xs[2 * a.n + jl] : 0.0f, qx, qy, qz) <= sc.eps2;
          if (ballot(hit)) {
            if (hit && !known_same_set(labels, jl, r)) uf_union(labels, r, jl, a.info);
            int nr = 0;
            if (lane == 0) nr = uf_find(labels, r, a.info);
            r = __shfl(nr, 0);
          }
          return false;
        }, labels, r);
      }
    return;
  }
  if (!packet) {  // spread out: every query walks on its own
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      if (!mine[s]) continue;
      const int i = idx[s];
      const Query qs = q[s];
      const Scope sc = scope_of<B>(a, m, i);
      int rs = root[s];
      traverse<D, true>(a.t, m, sc, qs, i, a.info, [&](int j) {
        if (!near<D>(a.xs, a.n, j, qs, sc.eps2)) return false;
        if (!(ALL_CORE || a.core[j])) return false;
        if (!known_same_set(labels, j, rs)) rs = uf_union(labels, rs, j, a.info);
        return false;
      });
    }
    return;
  }
  const float eps2 = ps.eps2;

  // Phase A: pairs inside the packet. Skipped when every query is already in one
  // set (the curve-neighbour unions usually see to that): its pairs would then
  // only join a set to itself.
  bool split = false;
#pragma unroll
  for (int s = 0; s < Q; ++s)
    if (mine[s]) root[s] = uf_find(labels, root[s], a.info);
  {
    int r0 = 0;
#pragma unroll
    for (int s = 0; s < Q; ++s)
      if (s == first_slot) r0 = root[s];
    r0 = __shfl(r0, fl);
#pragma unroll
    for (int s = 0; s < Q; ++s) split |= mine[s] && root[s] != r0;
  }
  const bool phase_a = ballot(split) != 0;
#pragma unroll
  for (int ks = 0; ks < Q && phase_a; ++ks) {
    for (int kl = 0; kl < 64; ++kl) {
      if (!((mm[ks] >> kl) & 1)) continue;
      const int jk = static_cast<int>(base) + ks * 64 + kl;
      const float px = readlane_f(q[ks].x, kl), py = readlane_f(q[ks].y, kl), pz = readlane_f(q[ks].z, kl);
#pragma unroll
      for (int s = 0; s < Q; ++s)
        if (mine[s] && jk > idx[s] && dist2v<D>(px, py, pz, q[s].x, q[s].y, q[s].z) <= eps2 &&
            !known_same_set(labels, jk, root[s]))
          root[s] = uf_union(labels, root[s], jk, a.info);
    }
  }
#pragma unroll
  for (int s = 0; s < Q; ++s)
    if (mine[s]) root[s] = uf_find(labels, root[s], a.info);
  int rl = 0;
#pragma unroll
  for (int s = 0; s < Q; ++s)
    if (s == first_slot) rl = root[s];
  int r = __shfl(rl, fl);
  bool differ = false;
#pragma unroll
  for (int s = 0; s < Q; ++s) differ |= mine[s] && root[s] != r;
  const bool common = !ballot(differ);
  const int p1 = static_cast<int>(base) + 64 * Q - 1;

  uint32_t* stack = s_stack + (threadIdx.x >> 6) * kWideStack;
  // the buckets a step reaches are laid end to end over the lanes (one candidate
  // per lane), so a step costs a round per 64 candidates, not one per bucket
  traverse_box_wide_lanes<D, true>(a.t, m, ps, lo, hi, i0, a.packet_leaf, a.info, stack, [&](int jl) {
    float cx = 0.0f, cy = 0.0f, cz = 0.0f;
    int cc = 0, cl = 0;
    if (jl >= 0) {
      cx = a.xs[jl];
      cy = a.xs[a.n + jl];
      cz = D == 3 ? a.xs[2 * a.n + jl] : 0.0f;
      cc = (ALL_CORE || a.core[jl]) ? 1 : 0;
      cl = ancestor_compress(labels, jl);
    }
    // candidates that need a test, decided by each candidate's own lane: outside the
    // packet (its pairs are phase A's; j > i0 by the mask), core, and not already in
    // the packet's set (r may grow during the round; a candidate skipped for the
    // old r is in the new r's set too, sets only merge)
    const bool need = jl > p1 && cc && !(common && cl == r);
    if (!ballot(need)) return false;
    if (common) {
      // every lane tests its own candidate against the queries (register
      // broadcasts, until every candidate has one within eps), and the lanes
      // that reach one join the packet's set together rather than one by one
      bool reach = false;
#pragma unroll
      for (int s = 0; s < Q; ++s)
        for (uint64_t qm = mm[s]; qm && ballot(need && !reach); qm &= qm - 1) {
          const int kl = __ffsll(static_cast<unsigned long long>(qm)) - 1;
          reach |= need && dist2v<D>(cx, cy, cz, readlane_f(q[s].x, kl), readlane_f(q[s].y, kl),
                                     readlane_f(q[s].z, kl)) <= eps2;
        }
      if (ballot(reach)) {
        if (reach && !known_same_set(labels, jl, r)) uf_union(labels, r, jl, a.info);
        int nr = 0;
        if (lane == fl) nr = uf_find(labels, r, a.info);
        r = __shfl(nr, fl);
      }
      return false;
    }
    for (uint64_t km = ballot(need); km; km &= km - 1) {
      const int k = __ffsll(static_cast<unsigned long long>(km)) - 1;
      const int j = __builtin_amdgcn_readlane(jl, k);
      const int lj = __builtin_amdgcn_readlane(cl, k);
      const float px = readlane_f(cx, k), py = readlane_f(cy, k), pz = readlane_f(cz, k);
#pragma unroll
      for (int s = 0; s < Q; ++s)
        if (mine[s] && lj != root[s] && dist2v<D>(px, py, pz, q[s].x, q[s].y, q[s].z) <= eps2 &&
            !known_same_set(labels, j, root[s]))
          root[s] = uf_union(labels, root[s], j, a.info);
    }
    return false;
  }, labels, common ? r : -1);
}

// Border pass from the core pass's neighbour records (no walk): the smallest
// cluster id among the recorded core neighbours.
__global__ void k_border_rec(TravArgs a) {
  const int nr = min(*a.brec_n, a.brec_cap);
  const int64_t k = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, nr);
  if (k < 0 || k >= nr) return;
  const int i = a.brec_i[k];
  int best = 0x7fffffff;
#pragma unroll
  for (int t = 0; t < kRecNb; ++t) {
    const int j = a.brec_nb[k * kRecNb + t];
    if (j >= 0 && a.core[j]) {
      const int c = a.cid[a.labels[j]];
      best = c < best ? c : best;
    }
  }
  a.border[i] = best == 0x7fffffff ? -1 : best;
}

// Border pass over the listed queries: non-core points whose neighbours were
// not all recorded (the core pass wrote -1 for lone points, and the records
// cover the rest).
template <int D, bool B>
__global__ void k_border_fdb(TravArgs a) {
  const int nq = *a.qborder_n;
  const int64_t k = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, nq);
  if (k < 0 || k >= nq) return;
  const int i = a.qborder[k];
  const int m = tree_m(a.t);
  const Scope sc = scope_of<B>(a, m, static_cast<int>(i));
  const Query q = load_point<D>(a.xs, a.n, i);
  int best = 0x7fffffff;
  traverse<D, false>(a.t, m, sc, q, 0, a.info, [&](int j) {
    if (!a.core[j] || !near<D>(a.xs, a.n, j, q, sc.eps2)) return false;
    int c = a.cid[a.labels[j]];
    best = c < best ? c : best;
    return best == 0;
  });
  a.border[i] = best == 0x7fffffff ? -1 : best;
}

// --------------------------------------------------------------- DenseBox ----
// Primitive p covers sorted points [prim_start[p], prim_start[p] + |cnt|):
// cnt > 0 is a single point, cnt < 0 a dense cell (all core, one cluster).
// Points outside dense cells query one lane per point primitive (so
// wavefronts are full and in Morton order); a dense cell queries once, one
// wavefront per cell, whose 64 lanes test the cell's points together.

// A walk reads primitive r through its leaf record prim_lo[r] (see TravArgs):
// one 16-byte load gives a point primitive's coordinates and sorted index, or a
// dense cell's low corner and first point.
__device__ __forceinline__ int rec_index(float4 lr) { return __float_as_int(lr.w); }

template <int D>
__device__ __forceinline__ bool rec_point_near(float4 lr, const Query& q, float eps2) {
  return dist2v<D>(lr.x, lr.y, lr.z, q.x, q.y, q.z) <= eps2;
}

template <int D>
__device__ __forceinline__ bool cell_box_near(const TravArgs& a, int r, float4 lo, const Query& q, float eps2) {
  const float4 hi = a.prim_hi[r];
  return box_dist2<D>(q.x, q.y, q.z, lo.x, lo.y, lo.z, hi.x, hi.y, hi.z) <= eps2;
}

// Is every point of the dense cell with tight box [lo, hi] within eps of q, as the
// point-by-point test would decide? Per axis the corner farther from q (by the
// rounded difference) bounds every point's rounded difference, since rounded
// subtraction, squaring and addition are monotone; so the test at that corner,
// made with the same operations in the same order, holds for all of them.
template <int D>
__device__ __forceinline__ bool cell_within(float4 lo, float4 hi, const Query& q, float eps2) {
  const float cx = fabsf(lo.x - q.x) > fabsf(hi.x - q.x) ? lo.x : hi.x;
  const float cy = fabsf(lo.y - q.y) > fabsf(hi.y - q.y) ? lo.y : hi.y;
  const float cz = fabsf(lo.z - q.z) > fabsf(hi.z - q.z) ? lo.z : hi.z;
  return dist2v<D>(cx, cy, cz, q.x, q.y, q.z) <= eps2;
}

// The query of point primitive p (its record), or an idle lane's (mine false).
__device__ __forceinline__ void own_record(const TravArgs& a, int p, int m, bool& mine, int& i, Query& q) {
  const float4 lr = p >= 0 && p < m ? a.prim_lo[p] : make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
  mine = rec_index(lr) >= 0;
  i = mine ? rec_index(lr) : 0;
  q.x = lr.x;
  q.y = lr.y;
  q.z = lr.z;
}

// Is some point of the cell [sa, sa+na) within eps of p? (whole wavefront)
template <int D>
__device__ __forceinline__ bool cell_reaches_point(const float* __restrict__ xs, int64_t n, int sa, int na, float px,
                                                   float py, float pz, float eps2) {
  const int lane = lane_id();
  for (int base = 0; base < na; base += 64) {
    bool h = false;
    if (base + lane < na) {
      const int64_t j = sa + base + lane;
      h = dist2v<D>(xs[j], xs[n + j], D == 3 ? xs[2 * n + j] : 0.0f, px, py, pz) <= eps2;
    }
    if (ballot(h)) return true;
  }
  return false;
}

// Is some pair (a in cell A, b in cell B) within eps? (whole wavefront.) A's
// points are taken 64 at a time, keeping those within eps of B's box; B's
// points are loaded 64 at a time too, keeping those within eps of the box of
// the kept A points (box gaps never exceed point distances, so nothing that
// could pass is dropped), and each kept B point is tested against all kept A
// points at once.
template <int D>
__device__ __forceinline__ bool cells_touch(const float* __restrict__ xs, int64_t n, int sa, int na, int sb, int nb,
                                           float4 blo, float4 bhi, float eps2) {
  const int lane = lane_id();
  for (int base = 0; base < na; base += 64) {
    bool act = base + lane < na;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    if (act) {
      const int64_t j = sa + base + lane;
      ax = xs[j];
      ay = xs[n + j];
      az = D == 3 ? xs[2 * n + j] : 0.0f;
      act = box_dist2<D>(ax, ay, az, blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z) <= eps2;
    }
    if (!ballot(act)) continue;
    // an A point whose eps-ball holds B's whole tight box pairs with every B point
    if (ballot(act && cell_within<D>(blo, bhi, Query{ax, ay, az}, eps2))) return true;
    float lo[3] = {act ? ax : INFINITY, act ? ay : INFINITY, act ? az : INFINITY};
    float hi[3] = {act ? ax : -INFINITY, act ? ay : -INFINITY, act ? az : -INFINITY};
#pragma unroll
    for (int k = 0; k < D; ++k)
      for (int off = 32; off > 0; off >>= 1) {
        lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
        hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
      }
    if (D == 2) lo[2] = hi[2] = 0.0f;
    for (int bb = 0; bb < nb; bb += 64) {
      bool near_b = bb + lane < nb;
      float bx = 0.0f, by = 0.0f, bz = 0.0f;
      if (near_b) {
        const int64_t j = sb + bb + lane;
        bx = xs[j];
        by = xs[n + j];
        bz = D == 3 ? xs[2 * n + j] : 0.0f;
        near_b = box_dist2<D>(bx, by, bz, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]) <= eps2;
      }
      for (uint64_t bm = ballot(near_b); bm; bm &= bm - 1) {
        const int k = __ffsll(static_cast<unsigned long long>(bm)) - 1;
        const float px = readlane_f(bx, k), py = readlane_f(by, k), pz = readlane_f(bz, k);
        if (ballot(act && dist2v<D>(ax, ay, az, px, py, pz) <= eps2)) return true;
      }
    }
  }
  return false;
}

// Number of points of the cell [s, s+c) within eps of p, counted 64 at a time
// until at least `want` (whole wavefront).
template <int D>
__device__ __forceinline__ int cell_count_near(const float* __restrict__ xs, int64_t n, int s, int c, float px,
                                               float py, float pz, float eps2, int want) {
  const int lane = lane_id();
  int found = 0;
  for (int base = 0; base < c && found < want; base += 64) {
    bool h = false;
    if (base + lane < c) {
      const int64_t j = s + base + lane;
      h = dist2v<D>(xs[j], xs[n + j], D == 3 ? xs[2 * n + j] : 0.0f, px, py, pz) <= eps2;
    }
    found += __popcll(ballot(h));
  }
  return found;
}

// Resumable per-lane walk, one primitive (or one internal node) per step, so
// that a wavefront can pause between steps: the sparse-point kernels below run
// their lanes in lock-step and, whenever some lanes have reached a dense cell,
// scan each such cell with the whole wavefront (64 points per ballot) instead
// of one lane looping over hundreds of points.
struct Walk {
  uint32_t node;  // next node to examine, kEnd when finished
  int cur, end;   // pending bucket primitives [cur, end]; empty when cur > end
  int last;       // last primitive of the scope
  uint32_t steps;  // remaining step budget (see traverse()); 2m + 2 <= 2^31
};

template <bool MASKED>
__device__ __forceinline__ void walk_init(Walk& w, int m, const Scope& sc, int mask, bool on) {
  w.cur = 1;
  w.end = 0;
  w.last = sc.end;
  w.steps = 2u * static_cast<uint32_t>(m) + 2u;
  if (!on || m <= 0 || (MASKED && mask >= sc.end)) w.node = kEnd;
  else w.node = sc.start;
}

__device__ __forceinline__ bool walk_done(const Walk& w) { return w.node == kEnd && w.cur > w.end; }

// A box query (every point of [lo, hi]); walk_step takes it or a point.
struct BoxQ {
  float lo[3], hi[3];
};

template <int D>
__device__ __forceinline__ float node_gap2(const Query& q, float4 a, float4 b) {
  return box_dist2<D>(q.x, q.y, q.z, a.x, a.y, a.z, b.x, b.y, b.z);
}
template <int D>
__device__ __forceinline__ float node_gap2(const BoxQ& q, float4 a, float4 b) {
  return boxbox_dist2<D>(q.lo, q.hi, a.x, a.y, a.z, b.x, b.y, b.z);
}

template <int D, bool MASKED, typename QT>
__device__ __forceinline__ int walk_step(Walk& w, const TreeView& t, int m, const QT& q, float eps2, int mask,
                                         uint32_t* info) {
  if (w.cur <= w.end) return w.cur++;
  const uint32_t node = w.node;
  if (node == kEnd) return -1;
  if (w.steps-- == 0) {
    atomicOr(info, kInternalBit);
    w.node = kEnd;
    return -1;
  }
  if (node & kLeaf) {
    const int l = static_cast<int>(node & ~kLeaf);
    if (l >= m) {
      atomicOr(info, kInternalBit);
      w.node = kEnd;
      return -1;
    }
    w.node = l >= w.last ? kEnd : static_cast<uint32_t>(t.leaf_rope[l]);
    return l;
  }
  if (node >= static_cast<uint32_t>(m - 1)) {
    atomicOr(info, kInternalBit);
    w.node = kEnd;
    return -1;
  }
  const float4 a = t.node_a[kNodeStride * size_t(node)];
  const float4 b = t.node_b[kNodeStride * size_t(node)];
  const uint32_t esc = static_cast<uint32_t>(t.rope[node]);  // loaded with the node
  const int k = static_cast<int>(node);
  const int o = __float_as_int(a.w), g = __float_as_int(b.w);
  const int first = o < k ? o : k, last = o > k ? o : k;
  if (node_gap2<D>(q, a, b) > eps2) {
    w.node = last >= w.last ? kEnd : esc;
    return -1;
  }
  if (first < 0 || last >= m || g < first || g >= last) {
    atomicOr(info, kInternalBit);
    w.node = kEnd;
    return -1;
  }
  if (last - first < t.leaf_size) {
    w.cur = (MASKED && first <= mask) ? mask + 1 : first;
    w.end = last;
    w.node = last >= w.last ? kEnd : esc;
    return w.cur <= w.end ? w.cur++ : -1;
  }
  if (MASKED && g <= mask)
    w.node = last == g + 1 ? (kLeaf | static_cast<uint32_t>(g + 1)) : static_cast<uint32_t>(g + 1);
  else
    w.node = first == g ? (kLeaf | static_cast<uint32_t>(g)) : static_cast<uint32_t>(g);
  return -1;
}

// ---- isolated points (one cloud, DenseBox, 32-bit grid keys) --------------------
// Before the core walks, a point primitive that has no neighbour but itself is
// settled by an occupancy map of the grid cells (side eps/sqrt(d)): one bit per
// cell, in 64-bit words per brick of 4x4x4 cells (3D) or 8x8 (2D). Bricks follow
// the Morton order, so a brick is the grid key without its lowest 6 bits; inside
// a brick, local cell (x, y, z) is bit x*16 + y*4 + z (3D) or x*8 + y (2D). A word
// is written only for an occupied brick, which a table of one bit per brick marks
// (the table is cleared each call, the words never are).
template <int D>
constexpr int kBrickShift = D == 3 ? 2 : 3;  // local coordinate bits per axis

template <int D>
__device__ __forceinline__ int brick_bit(uint32_t code) {  // from the code's lowest 6 bits
  if constexpr (D == 3) {
    const uint32_t z = (code & 1u) | ((code >> 2) & 2u);
    const uint32_t y = ((code >> 1) & 1u) | ((code >> 3) & 2u);
    const uint32_t x = ((code >> 2) & 1u) | ((code >> 4) & 2u);
    return static_cast<int>(x * 16 + y * 4 + z);
  } else {
    const uint32_t y = (code & 1u) | ((code >> 1) & 2u) | ((code >> 2) & 4u);
    const uint32_t x = ((code >> 1) & 1u) | ((code >> 2) & 2u) | ((code >> 3) & 4u);
    return static_cast<int>(x * 8 + y);
  }
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int off) {
  const uint32_t lo = static_cast<uint32_t>(__shfl_up(static_cast<int>(v), off));
  const uint32_t hi = static_cast<uint32_t>(__shfl_up(static_cast<int>(v >> 32), off));
  return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int off) {
  const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off));
  const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v >> 32), off));
  return (uint64_t(hi) << 32) | lo;
}

// A brick word is written once, by the wavefront holding the brick's first
// primitive: a segmented OR over the wavefront's 64 primitives, and for its last
// brick the following primitives of the same brick, read 64 at a time.
// It also clears the list counters of k_lone_filter, which runs after it.
// Primitive keys are 64-bit words; the isolated-point test runs on grids keyed in
// 32 bits, so only the low word carries the key.
__device__ __forceinline__ uint32_t key32(const uint64_t* __restrict__ pkey, int64_t p) {
  return static_cast<uint32_t>(pkey[p]);
}

// Clears the occupancy words (as many as the plan asks for; none when the test
// does not run).
__global__ __launch_bounds__(256) void k_lone_clear(const GridPlan* __restrict__ plan, uint64_t* __restrict__ bits) {
  if (!plan->lone_on) return;
  const int64_t words = (plan->lone_words + 63) / 64;  // the brick table, 64 brick bits per word
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < words; i += int64_t(gridDim.x) * blockDim.x)
    bits[i] = 0ull;
}

template <int D>
__global__ __launch_bounds__(256) void k_lone_bits(const uint64_t* __restrict__ pkey, const int* __restrict__ d_m,
                                                   const GridPlan* __restrict__ plan, uint64_t* __restrict__ bits,
                                                   uint32_t* __restrict__ table, int* __restrict__ list_n) {
  if (!plan->lone_on) return;
  if (blockIdx.x == 0 && threadIdx.x < kNumXcd) list_n[threadIdx.x] = 0;
  const int m = *d_m;
  const int lane = lane_id();
  // a wavefront per 64 primitives, over a grid-stride loop (uniform per wavefront)
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t p0 = (blockIdx.x * int64_t(blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; p0 < m; p0 += waves * 64) {
    const int64_t p = p0 + lane;
    const bool valid = p < m;
    const uint32_t code = valid ? key32(pkey, p) : 0xffffffffu;
    const uint32_t word = code >> 6;  // invalid lanes: above every valid brick
    const uint32_t prevw = static_cast<uint32_t>(__shfl_up(static_cast<int>(word), 1));
    const uint32_t nextw = static_cast<uint32_t>(__shfl_down(static_cast<int>(word), 1));
    const bool head = lane == 0 || word != prevw;
    // segmented inclusive OR: the last lane of a run of equal bricks holds the run's bits
    uint64_t v = valid ? (1ull << brick_bit<D>(code)) : 0ull;
    bool f = head;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t u = shfl_up_u64(v, off);
      const bool g = __shfl_up(static_cast<int>(f), off) != 0;
      if (lane >= off && !f) {
        v |= u;
        f = g;
      }
    }
    const uint32_t w0 = static_cast<uint32_t>(__shfl(static_cast<int>(word), 0));
    // the wavefront's first run may continue a brick begun by the previous
    // wavefront, which then writes it
    const bool continued = p0 > 0 && (key32(pkey, p0 - 1) >> 6) == w0;
    const bool in_first_run = __popcll(ballot(head) & (lanemask_lt() | (1ull << lane))) == 1;
    const uint32_t w63 = static_cast<uint32_t>(__shfl(static_cast<int>(word), 63));
    uint64_t extra = 0;
    // lane 63 is valid and its run may go on past this wavefront; only the
    // wavefront that writes that brick reads ahead
    if (p0 + 64 < m && !(continued && w63 == w0)) {
      for (int64_t b = p0 + 64; b < m; b += 64) {
        const int64_t q = b + lane;
        const uint32_t c2 = q < m ? key32(pkey, q) : 0xffffffffu;
        const bool in = q < m && (c2 >> 6) == w63;
        uint64_t x = in ? (1ull << brick_bit<D>(c2)) : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x |= shfl_xor_u64(x, off);
        extra |= x;
        if (!((ballot(in) >> 63) & 1)) break;  // codes are sorted: the run ended in this chunk
      }
    }
    const bool tail = valid && (lane == 63 || nextw != word);
    const bool writes = tail && !(continued && in_first_run);
    if (writes) bits[word] = v | (lane == 63 ? extra : 0ull);
    // mark the written bricks in the table: the writers' bricks rise with the lanes,
    // so those sharing a table word are consecutive; one atomic per table word
    const uint32_t tw = word >> 5;
    for (uint64_t wm = ballot(writes); wm;) {
      const int L = __ffsll(static_cast<unsigned long long>(wm)) - 1;
      const uint32_t t0 = static_cast<uint32_t>(__shfl(static_cast<int>(tw), L));
      const uint64_t grp = ballot(writes && tw == t0);
      uint32_t mbits = (writes && tw == t0) ? 1u << (word & 31) : 0u;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) mbits |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(mbits), off));
      if (lane == L) atomicOr(table + t0, mbits);
      wm &= ~grp;
    }
  }
}

__device__ __forceinline__ uint32_t compact_every(uint32_t x, int d) {  // inverse of the Morton spread
  if (d == 3) {
    x &= 0x09249249u;
    x = (x | (x >> 2)) & 0x030c30c3u;
    x = (x | (x >> 4)) & 0x0300f00fu;
    x = (x | (x >> 8)) & 0xff0000ffu;
    x = (x | (x >> 16)) & 0x000003ffu;
  } else {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0f0f0f0fu;
    x = (x | (x >> 4)) & 0x00ff00ffu;
    x = (x | (x >> 8)) & 0x0000ffffu;
  }
  return x;
}

__device__ __forceinline__ uint32_t spread_every(uint32_t x, int d) {  // Morton spread of one coordinate
  if (d == 3) {
    x &= 0x000003ffu;
    x = (x | (x << 16)) & 0xff0000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
  } else {
    x &= 0x0000ffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
  }
  return x;
}

// A point primitive is isolated when no other primitive shares its cell (they
// would be next to it in key order) and no occupied cell lies within reach of it:
// in cell units, the per-axis gaps between the point's coordinate t = (x - lo) /
// side and a cell's interval, summed in squares, exceed plan->reach^2, where reach
// is eps / side plus a slack covering the rounding of t (computed as the key
// kernel computes it) for both points. A neighbour j of the point (the fp32 test
// true) is within eps (1 + 2^-22) per axis; its cell's gap vector is bounded by
// |t_j - t| per axis, whose norm the slack covers, so its cell is within reach.
// Conservative: a false answer only means "walk it". Reach is below 2, so the
// reachable cells lie within 2 per axis: at most 2^d brick words per query, each
// current only when its bit in the table is set.

// Bits of a brick whose coordinate on axis a lies in [l, h] (local, l <= h).
template <int D>
__device__ __forceinline__ uint64_t axis_bits(int a, int l, int h) {
  if constexpr (D == 3) {
    if (a == 0) return (~0ull >> (48 - 16 * h)) & (~0ull << (16 * l));
    if (a == 1) return uint64_t((0xffffu >> (12 - 4 * h)) & (0xffffu << (4 * l)) & 0xffffu) * 0x0001000100010001ull;
    return uint64_t((0xfu >> (3 - h)) & (0xfu << l) & 0xfu) * 0x1111111111111111ull;
  } else {
    if (a == 0) return (~0ull >> (56 - 8 * h)) & (~0ull << (8 * l));
    return uint64_t((0xffu >> (7 - h)) & (0xffu << l) & 0xffu) * 0x0101010101010101ull;
  }
}

// Gap of coordinate t (its own cell c) to the interval of cell `cell`, in cell units.
__device__ __forceinline__ float cell_gap(float t, int c, int cell) {
  return cell == c ? 0.0f : (cell > c ? static_cast<float>(cell) - t : t - static_cast<float>(cell + 1));
}

template <int D>
__device__ __forceinline__ bool isolated(const uint64_t* __restrict__ pkey, int m, int p, float4 pt,
                                         const GridPlan& g, const float* lo_b, const uint64_t* __restrict__ words,
                                         const uint32_t* __restrict__ table) {
  // Straight-line on purpose: the three keys are loaded together, then every
  // brick's table bit and word together (a word of an unmarked brick is stale
  // and discarded), so a query waits for two memory round trips, not one per
  // brick. Bricks outside the grid load brick 0 and are masked out.
  const uint32_t key = key32(pkey, p);
  const uint32_t kprev = key32(pkey, p > 0 ? p - 1 : p);
  const uint32_t knext = key32(pkey, p + 1 < m ? p + 1 : p);
  const bool shared = (p > 0 && kprev == key) || (p + 1 < m && knext == key);
  constexpr int S = kBrickShift<D>, W = 1 << S;
  constexpr int NB = D == 3 ? 8 : 4;  // bricks that can hold cells within 2 per axis
  const float xv[3] = {pt.x, pt.y, pt.z};
  float t[3] = {0.0f, 0.0f, 0.0f};
  int c[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    t[a] = fmaxf((xv[a] - lo_b[a]) * g.inv_h[a], 0.0f);  // as the key kernel computes it
    c[a] = static_cast<int>(compact_every(key >> (D - 1 - a), D));
    lo[a] = c[a] >= 2 ? c[a] - 2 : 0;
    hi[a] = min(c[a] + 2, static_cast<int>(g.ncell[a]) - 1);
  }
  uint32_t bidx[NB];
  uint64_t bbox[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    const int br[3] = {(lo[0] >> S) + (n >> (D - 1)), (lo[1] >> S) + ((n >> (D - 2)) & 1), (lo[2] >> S) + (n & 1)};
    bool use = br[0] <= (hi[0] >> S) && br[1] <= (hi[1] >> S);
    if (D == 3) use = use && br[2] <= (hi[2] >> S);
    uint32_t b = 0;
    uint64_t box = ~0ull;  // the brick's cells within 2 per axis
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int base = br[a] << S;
      box &= axis_bits<D>(a, max(lo[a], base) - base, min(hi[a], base + W - 1) - base);
      b |= spread_every(static_cast<uint32_t>(br[a]), D) << (D - 1 - a);
    }
    bidx[n] = use ? b : 0u;
    bbox[n] = use ? box : 0ull;
  }
  uint32_t tw[NB];
  uint64_t ww[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    tw[n] = table[bidx[n] >> 5];
    ww[n] = words[bidx[n]];
  }
  const uint32_t own_brick = key >> 6;
  const int own_bit = brick_bit<D>(key);
  const float r2 = g.reach * g.reach;
  bool near = shared;
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    uint64_t occ = (tw[n] >> (bidx[n] & 31)) & 1u ? ww[n] & bbox[n] : 0ull;
    if (bidx[n] == own_brick) occ &= ~(1ull << own_bit);
    // the occupied cells among them (usually none, or a few): exact reach test
    const int bx = static_cast<int>(compact_every(bidx[n] >> (D - 1), D)) << S;
    const int by = static_cast<int>(compact_every(bidx[n] >> (D - 2), D)) << S;
    const int bz = D == 3 ? static_cast<int>(compact_every(bidx[n], D)) << S : 0;
    for (; occ && !near; occ &= occ - 1) {
      const int bit = __ffsll(static_cast<unsigned long long>(occ)) - 1;
      const int lx = D == 3 ? bit >> 4 : bit >> 3;
      const int ly = D == 3 ? (bit >> 2) & 3 : bit & 7;
      const int lz = D == 3 ? bit & 3 : 0;
      const float gx = cell_gap(t[0], c[0], bx + lx);
      const float gy = cell_gap(t[1], c[1], by + ly);
      const float gz = D == 3 ? cell_gap(t[2], c[2], bz + lz) : 0.0f;
      near = gx * gx + gy * gy + gz * gz <= r2;
    }
  }
  return !near;
}

// A workgroup tests kLoneRounds x 256 consecutive primitives and lists the ones
// left for the core pass with one atomic (a counter taken by many workgroups is
// the cost to keep low), in primitive order within the workgroup. The primitives
// are cut into kNumXcd segments of lone_segment(m) (a multiple of a workgroup's
// share); segment s has its own counter and lists into list[s * segment ...], which
// never passes its own primitive range, so the list needs m entries. The core pass
// gives segment s to the workgroups of XCD s: each XCD walks one contiguous range
// of the curve, as it does without the test.
constexpr int kLoneRounds = 4;

__device__ __forceinline__ int64_t lone_segment(int m) {
  const int64_t share = kLoneRounds * 256;
  return ((m + kNumXcd - 1) / kNumXcd + share - 1) / share * share;
}

template <int D>
__global__ __launch_bounds__(256) void k_lone_filter(TravArgs a, const uint64_t* __restrict__ pkey,
                                                     const GridPlan* __restrict__ plan,
                                                     const uint64_t* __restrict__ words,
                                                     const uint32_t* __restrict__ table,
                                                     const uint32_t* __restrict__ bounds, int* __restrict__ list,
                                                     int* __restrict__ list_n) {
  __shared__ int s_cnt[kLoneRounds * 4 + 1];
  if (!plan->lone_on) return;
  const GridPlan gp = *plan;
  float lo_b[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < D; ++k) lo_b[k] = ord2f(bounds[k]);
  const int m = tree_m(a.t);
  const int64_t base = blockIdx.x * int64_t(kLoneRounds * 256);
  if (base >= m) return;  // whole workgroup
  const int64_t segment = lone_segment(m);
  const int seg = static_cast<int>(base / segment);  // a workgroup lies in one segment
  const int w = threadIdx.x >> 6;
  uint32_t keep = 0;  // bit r: primitive of round r is listed
  for (int r = 0; r < kLoneRounds; ++r) {
    const int64_t p = base + r * 256 + threadIdx.x;
    bool query = false, lone = false;
    int i = 0;
    if (p < m) {
      // the test's loads do not wait for the record (a dense cell's answer is discarded)
      const float4 lr = a.prim_lo[p];
      const bool iso = isolated<D>(pkey, m, static_cast<int>(p), lr, gp, lo_b, words, table);
      i = rec_index(lr);
      query = i >= 0;
      lone = query && iso;
    }
    if (lone) {
      a.core[i] = 0;
      a.lone[i] = 1;
      a.border[i] = -1;
    }
    const bool listed = query && !lone;
    keep |= listed ? 1u << r : 0u;
    const uint64_t bal = ballot(listed);
    if (lane_id() == 0) s_cnt[r * 4 + w] = __popcll(bal);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < kLoneRounds * 4; ++k) {
      const int c = s_cnt[k];
      s_cnt[k] = tot;
      tot += c;
    }
    s_cnt[kLoneRounds * 4] = tot ? atomicAdd(list_n + seg, tot) : 0;
  }
  __syncthreads();
  const int64_t start = s_cnt[kLoneRounds * 4] + seg * segment;
  for (int r = 0; r < kLoneRounds; ++r) {
    const bool listed = (keep >> r) & 1u;
    const uint64_t bal = ballot(listed);
    if (listed)
      list[start + s_cnt[r * 4 + w] + __popcll(bal & lanemask_lt())] = static_cast<int>(base + r * 256 + threadIdx.x);
  }
}

// Core pass for points outside dense cells. Each lane walks for kCoreQ
// neighbouring point primitives (kCoreQ k + t for lane k of the index space).
// Two walks per lane keep more node loads in flight, but a wavefront then waits
// for the longest of 128 walks and the 8M-point set fills fewer wavefronts than
// the chip has slots: measured slower (0.55 vs 0.47 ms), so one.
constexpr int kCoreQ = 1;

template <int D, bool B>
__global__ void k_core_dbx(TravArgs a) {
  __shared__ int s_w[17];
  extern __shared__ int s_rec[];  // kCoreQ tables of kRecNb * blockDim.x
  const int m = tree_m(a.t);
  const int lane = lane_id();
  // the grid is sized for n queries; a workgroup past the m primitives leaves
  // at once (uniformly, before any barrier)
  static_assert(kCoreQ == 1, "a listed query is one primitive");
  // listed queries: XCD x (workgroup index mod kNumXcd) takes segment x of the list
  const int xcd = static_cast<int>(blockIdx.x % kNumXcd);
  const bool listed = a.core_list && (!a.lone_on || *a.lone_on);
  const int* qlist = listed ? a.core_list + xcd * lone_segment(m) : nullptr;
  const int64_t total = listed ? a.core_qn[xcd] : (m + kCoreQ - 1) / kCoreQ;
  const int64_t k0 = listed ? int64_t(blockIdx.x / kNumXcd) * blockDim.x
                            : xcd_spread(blockIdx.x, blockDim.x, 0, total);
  if (k0 < 0 || k0 >= total) return;
  const int64_t k = listed ? k0 + threadIdx.x : xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, total);
  int p[kCoreQ], i[kCoreQ], cnt[kCoreQ];
  bool mine[kCoreQ], active[kCoreQ];
  Scope sc[kCoreQ];
  Query q[kCoreQ];
  NbRec rec[kCoreQ];
  Walk w[kCoreQ];
#pragma unroll
  for (int t = 0; t < kCoreQ; ++t) {
    p[t] = k < 0 || k >= total ? -1 : (qlist ? qlist[k] : static_cast<int>(k * kCoreQ + t));
    own_record(a, p[t], m, mine[t], i[t], q[t]);  // dense cells are core by construction
    sc[t] = scope_of<B>(a, m, i[t]);
    cnt[t] = 0;
    rec_init(rec[t], s_rec + t * kRecNb * blockDim.x);
  }
#pragma unroll
  for (int t = 0; t < kCoreQ; ++t) {
    walk_init<false>(w[t], m, sc[t], 0, mine[t]);
    active[t] = mine[t] && !walk_done(w[t]);
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int t = 0; t < kCoreQ; ++t) any |= active[t];
    if (!ballot(any)) break;
    int pend[kCoreQ], pcnt[kCoreQ];  // a dense cell to scan: its first point and its size
#pragma unroll
    for (int t = 0; t < kCoreQ; ++t) {
      pend[t] = -1;
      pcnt[t] = 0;
      if (active[t]) {
        const int r = walk_step<D, false>(w[t], a.t, m, q[t], sc[t].eps2, 0, a.info);
        if (r >= 0) {
          const float4 lr = a.prim_lo[r];
          const int s = rec_index(lr);
          if (s >= 0) {
            if (rec_point_near<D>(lr, q[t], sc[t].eps2)) {
              ++cnt[t];
              if (s != i[t]) rec_add(rec[t], s);
            }
          } else {
            const float4 hr = a.prim_hi[r];
            if (box_dist2<D>(q[t].x, q[t].y, q[t].z, lr.x, lr.y, lr.z, hr.x, hr.y, hr.z) <= sc[t].eps2) {
              if (cell_within<D>(lr, hr, q[t], sc[t].eps2)) {  // counted whole, no scan
                cnt[t] += __float_as_int(hr.w);
                rec_add(rec[t], s);  // s == cell_ref(first point)
              } else {  // both from the records already loaded: the scan starts with the points
                pend[t] = ref_point(s);
                pcnt[t] = __float_as_int(hr.w);
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kCoreQ; ++t) {
      for (uint64_t pm = ballot(pend[t] >= 0); pm; pm &= pm - 1) {
        const int L = __ffsll(static_cast<unsigned long long>(pm)) - 1;
        const int s = __shfl(pend[t], L);
        const int want = __shfl(sc[t].min_pts - cnt[t], L);
        const int found = cell_count_near<D>(a.xs, a.n, s, __shfl(pcnt[t], L), __shfl(q[t].x, L), __shfl(q[t].y, L),
                                             __shfl(q[t].z, L), readlane_f(sc[t].eps2, L), want);
        if (lane == L && found > 0) {
          cnt[t] += found;
          rec_add(rec[t], cell_ref(s));  // a dense cell: all core, one cluster; its first point stands for it
        }
      }
      if (active[t] && (cnt[t] >= sc[t].min_pts || walk_done(w[t]))) active[t] = false;
    }
  }
#pragma unroll
  for (int t = 0; t < kCoreQ; ++t) core_epilogue(a, mine[t], i[t], p[t], cnt[t], sc[t].min_pts, rec[t], s_w);
}

// Main phase, points outside dense cells: pairs with primitives above their own.
// One lane per point primitive; lanes whose point is not a query stay idle.
// (Compacting the few core queries into full wavefronts was slower: their
// wavefront-wide cell scans then run on too few wavefronts to fill the chip.)
// Canonical labels: when a wavefront's core queries lie in a box at most
// kPointsPacketExt eps wide (and, in a batch, in one cloud), they walk as one
// packet: one lane-parallel wide walk over the box reaches every primitive above
// the smallest query within eps of any query; each candidate is broadcast and
// every lane keeps the pairs above its own primitive, so the unions are those of
// the per-lane walks. Queries around a dense clump otherwise each walk most of
// the clump's subtree one node per step.
constexpr float kPointsPacketExt = 8.0f;
constexpr int kPointsFewQueries = 32;   // at most this many queries ...
constexpr float kPointsFewExt = 32.0f;  // ... form a packet up to this many eps wide

template <int D, bool ALL_CORE, bool FIRST, bool B>
__global__ void k_main_dbx_points(TravArgs a) {
  extern __shared__ uint32_t s_pstack[];  // kWideStack entries per wavefront
  const int m = tree_m(a.t);
  const int lane = lane_id();
  const int64_t p0 = xcd_spread(blockIdx.x, blockDim.x, 0, m);
  if (p0 < 0 || p0 >= m) return;  // the grid is sized for n; past the primitives
  const int p = static_cast<int>(xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, m));
  bool pt;
  int i;
  Query q;
  own_record(a, p, m, pt, i, q);
  const bool ci = pt && (ALL_CORE || a.core[i]);
  const bool mine = pt && (ci || (FIRST && !is_lone(a, i)));
  const Scope sc = scope_of<B>(a, m, i);
  int* labels = a.labels;
  // the core pass may already have joined i to dense cells it reaches
  int root = mine && ci ? uf_find(labels, i, a.info) : i;
  if (!FIRST) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (mine) {
      lo[0] = hi[0] = q.x;
      lo[1] = hi[1] = q.y;
      lo[2] = hi[2] = q.z;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
      for (int off = 32; off > 0; off >>= 1) {
        lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
        hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
      }
    const uint64_t mm = ballot(mine);
    if (!mm) return;
    const int fl = __ffsll(static_cast<unsigned long long>(mm)) - 1;
    const int i0 = __shfl(i, fl), pmin = __shfl(p, fl);  // primitives rise with the lanes
    const Scope ps = scope_of<B>(a, m, i0);
    const bool other_cloud = B && mine && cloud_of(a, i) != cloud_of(a, i0);
    float ext = fmaxf(hi[0] - lo[0], hi[1] - lo[1]);
    if (D == 3) ext = fmaxf(ext, hi[2] - lo[2]);
    // a few queries spread wider still walk as one packet: their per-lane walks
    // would each cross the clumps in between on their own
    const float ext_max = __popcll(mm) <= kPointsFewQueries ? kPointsFewExt : kPointsPacketExt;
    if (!ballot(other_cloud) && ext * ext <= ext_max * ext_max * ps.eps2) {
      const float eps2 = ps.eps2;
      // Phase A: pairs of this wavefront's own queries (every core point primitive
      // in its range is a query), each joined from its lower primitive.
      for (uint64_t km = mm; km; km &= km - 1) {
        const int kl = __ffsll(static_cast<unsigned long long>(km)) - 1;
        const int jk = __shfl(i, kl);
        const float px = readlane_f(q.x, kl), py = readlane_f(q.y, kl), pz = readlane_f(q.z, kl);
        if (mine && lane < kl && dist2v<D>(px, py, pz, q.x, q.y, q.z) <= eps2 && !known_same_set(labels, jk, root))
          root = uf_union(labels, root, jk, a.info);
      }
      if (mine) root = uf_find(labels, root, a.info);
      int r = __shfl(root, fl);
      bool common = !ballot(mine && root != r);
      const int plast = __shfl(p, 63);  // point primitives up to here are this wavefront's (phase A)
      uint32_t* stack = s_pstack + (threadIdx.x >> 6) * kWideStack;
      traverse_box_wide_lanes<D>(a.t, m, ps, lo, hi, pmin, a.t.leaf_size, a.info, stack, [&](int rr) {
        float4 lr = make_float4(0.0f, 0.0f, 0.0f, 0.0f), hr = lr;
        bool hit = false;
        int anc = -1;
        if (rr >= 0) {
          lr = a.prim_lo[rr];
          const int v = rec_index(lr);
          if (v >= 0) {
            hit = rr > plast && (ALL_CORE || a.core[v]) &&
                  box_dist2<D>(lr.x, lr.y, lr.z, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]) <= eps2;
          } else {
            hr = a.prim_hi[rr];
            hit = boxbox_dist2<D>(lo, hi, lr.x, lr.y, lr.z, hr.x, hr.y, hr.z) <= eps2;
          }
          if (hit) anc = ancestor_compress(labels, ref_point(v));
        }
        const bool is_pt = rec_index(lr) >= 0;
        if (common) {
          // Points, all at once: every lane tests its own candidate against all
          // queries (register broadcasts), then the lanes that reach one join
          // the packet's set in parallel.
          const bool cand = hit && is_pt && anc != r;
          if (ballot(cand)) {
            bool reach = false;
            for (uint64_t qm = mm; qm; qm &= qm - 1) {
              const int kl = __ffsll(static_cast<unsigned long long>(qm)) - 1;
              reach |= cand && dist2v<D>(lr.x, lr.y, lr.z, readlane_f(q.x, kl), readlane_f(q.y, kl),
                                         readlane_f(q.z, kl)) <= eps2;
            }
            if (ballot(reach)) {
              if (reach && !known_same_set(labels, rec_index(lr), r)) uf_union(labels, r, rec_index(lr), a.info);
              int nr = 0;
              if (lane == fl) nr = uf_find(labels, r, a.info);
              r = __shfl(nr, fl);
              root = r;
            }
          }
        }
        // cells, and points when the queries are in several sets: one at a time
        for (uint64_t vm = ballot(hit && !(common && (is_pt || anc == r))); vm; vm &= vm - 1) {
          const int k = __ffsll(static_cast<unsigned long long>(vm)) - 1;
          const int rk = __builtin_amdgcn_readlane(rr, k);
          const int v = __builtin_amdgcn_readlane(rec_index(lr), k);
          const int j = ref_point(v);
          const int ak = __builtin_amdgcn_readlane(anc, k);
          const float px = readlane_f(lr.x, k), py = readlane_f(lr.y, k), pz = readlane_f(lr.z, k);
          if (common && ak == r) continue;  // joined by an earlier candidate of this walk
          if (v >= 0) {  // a core point above every query of the wavefront (queries in several sets)
            if (mine && ak != root && dist2v<D>(px, py, pz, q.x, q.y, q.z) <= eps2 && !known_same_set(labels, j, root))
              root = uf_union(labels, root, j, a.info);
            continue;
          }
          // a dense cell: one of its points within eps of a query suffices
          const float ux = readlane_f(hr.x, k), uy = readlane_f(hr.y, k), uz = readlane_f(hr.z, k);
          const int nk = __builtin_amdgcn_readlane(__float_as_int(hr.w), k);  // the cell's size
          const bool nb = mine && rk > p && (common || ak != root) &&
                          box_dist2<D>(q.x, q.y, q.z, px, py, pz, ux, uy, uz) <= eps2 &&
                          (common || !known_same_set(labels, j, root));
          if (common && ballot(nb) && known_same_set(labels, j, r)) continue;
          // a query whose eps-ball holds the whole cell reaches it without a scan
          const bool full = nb && cell_within<D>(make_float4(px, py, pz, 0.0f), make_float4(ux, uy, uz, 0.0f), q, eps2);
          if (common) {
            const uint64_t fm = ballot(full);
            if (fm) {
              const int L = __ffsll(static_cast<unsigned long long>(fm)) - 1;
              int nr = 0;
              if (lane == L) nr = uf_union(labels, r, j, a.info);
              r = __shfl(nr, L);
              root = r;
              continue;  // the whole packet is in one set with the cell now
            }
          } else if (full) {
            root = uf_union(labels, root, j, a.info);
          }
          for (uint64_t lm = ballot(nb && !full); lm; lm &= lm - 1) {
            const int L = __ffsll(static_cast<unsigned long long>(lm)) - 1;
            const bool reach = cell_reaches_point<D>(a.xs, a.n, j, nk, readlane_f(q.x, L),
                                                     readlane_f(q.y, L), readlane_f(q.z, L), eps2);
            if (common) {
              if (!reach) continue;
              int nr = 0;
              if (lane == L) nr = uf_union(labels, r, j, a.info);
              r = __shfl(nr, L);
              root = r;
              break;  // the whole packet is in one set with the cell now
            }
            if (lane == L && reach) root = uf_union(labels, root, j, a.info);
          }
        }
        return false;
      });
      return;
    }
  }
  Walk w;
  walk_init<true>(w, m, sc, p, mine);
  bool active = mine && !walk_done(w);
  while (ballot(active)) {
    int pend = -1;
    if (active) {
      const int r = walk_step<D, true>(w, a.t, m, q, sc.eps2, p, a.info);
      if (r >= 0) {
        const float4 lr = a.prim_lo[r];
        const int s = rec_index(lr);
        if (s >= 0) {
          if (rec_point_near<D>(lr, q, sc.eps2)) {
            const bool cj = ALL_CORE || a.core[s];
            if (ci && cj) {
              if (!known_same_set(labels, s, root)) root = uf_union(labels, root, s, a.info);
            } else if (FIRST && ci) {
              uf_claim(labels, s, i);
            } else if (FIRST && cj) {
              uf_claim(labels, i, s);
              active = false;  // i is a member now (by this or an earlier claim)
            }
          }
        } else if (cell_box_near<D>(a, r, lr, q, sc.eps2) && !(ci && known_same_set(labels, ref_point(s), root))) {
          pend = r;
        }
      }
    }
    // a dense cell: one of its points within eps suffices
    for (uint64_t pm = ballot(pend >= 0); pm; pm &= pm - 1) {
      const int L = __ffsll(static_cast<unsigned long long>(pm)) - 1;
      const int r = __shfl(pend, L);
      const int s = a.prim_start[r];
      const bool hit = cell_reaches_point<D>(a.xs, a.n, s, -a.prim_cnt[r], __shfl(q.x, L), __shfl(q.y, L),
                                             __shfl(q.z, L), readlane_f(sc.eps2, L));
      if (lane == L && hit) {
        if (ci) {
          root = uf_union(labels, root, s, a.info);
        } else if (FIRST) {
          uf_claim(labels, i, s);
          active = false;
        }
      }
    }
    if (active && walk_done(w)) active = false;
  }
}

// Main phase, dense cells, when they are few (see cells_lane_mode):
// one wavefront per cell A walks the tree once with A's box,
// over primitives above A; a dense neighbour B joins A's set if some pair is
// within eps, a core point if some point of A reaches it, and (first-claim
// mode) a non-core point is claimed the same way. Many cells go to
// k_main_dbx_cells_lane instead (the two kernels are launched together and each
// leaves the other's case alone).
constexpr int kCellsPerWaveMax = 65536;

// More than 65,536 dense cells (8 per wavefront of the 8192 below) go to the
// lane-per-cell kernel: measured faster there, for small cells (a batch of 4,096
// clouds: 13 vs 62 ms) and for large ones (a batch of 50 clouds of up to 2M
// points: 3 vs 8 ms); with fewer cells a wavefront per cell keeps more
// wavefronts busy (8M-point set, 20k cells: 0.3 vs 0.96 ms). Both kernels read
// the count.
__device__ __forceinline__ bool cells_lane_mode(const TravArgs& a) { return *a.d_ndense > kCellsPerWaveMax; }

template <int D, bool ALL_CORE, bool FIRST, bool B>
__global__ __launch_bounds__(256) void k_main_dbx_cells_wave(TravArgs a) {
  __shared__ uint32_t s_stack[4 * kWideStack];  // 256-thread workgroups
  uint32_t* stack = s_stack + (threadIdx.x >> 6) * kWideStack;
  const int nd = *a.d_ndense;
  if (cells_lane_mode(a)) return;
  const int m = tree_m(a.t);
  const int lane = lane_id();
  const int wave = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  int* labels = a.labels;
  // wavefront w takes a contiguous slice of the dense-cell list (filled in
  // roughly increasing key order), so neighbouring cells share an XCD's L2
  const int per = (nd + nwaves - 1) / nwaves;
  const int dbeg = wave * per, dend = min(nd, dbeg + per);
  for (int w = dbeg; w < dend; ++w) {
    const int A = a.dense_list[w];
    const int sa = a.prim_start[A], na = -a.prim_cnt[A];
    const Scope sc = scope_of<B>(a, m, sa);
    const float eps2 = sc.eps2;
    const float4 alo4 = a.prim_lo[A], ahi4 = a.prim_hi[A];
    const float alo[3] = {alo4.x, alo4.y, alo4.z}, ahi[3] = {ahi4.x, ahi4.y, ahi4.z};
    // the core pass may already have joined A to other sets
    int root = uf_find(labels, sa, a.info);
    traverse_box_wide_lanes<D>(a.t, m, sc, alo, ahi, A, a.t.leaf_size, a.info, stack, [&](int r) {
      // every lane loads its primitive's record and what decides a skip (core
      // flag, an ancestor near the root); candidates then go one after another
      float4 lr = make_float4(0.0f, 0.0f, 0.0f, 0.0f), hr = lr;
      bool hit = false, cj = false;
      int anc = -1;
      if (r >= 0) {
        lr = a.prim_lo[r];
        const int v = rec_index(lr);
        if (v >= 0) {
          hit = box_dist2<D>(lr.x, lr.y, lr.z, alo[0], alo[1], alo[2], ahi[0], ahi[1], ahi[2]) <= eps2;
        } else {
          hr = a.prim_hi[r];
          hit = boxbox_dist2<D>(alo, ahi, lr.x, lr.y, lr.z, hr.x, hr.y, hr.z) <= eps2;
        }
        if (hit) {
          const int j = ref_point(v);
          cj = v < 0 || ALL_CORE || a.core[j];  // dense cells are core
          anc = cj ? ancestor_compress(labels, j) : labels[j];
        }
      }
      for (uint64_t vm = ballot(hit && !(cj && anc == root)); vm; vm &= vm - 1) {
        const int k = __ffsll(static_cast<unsigned long long>(vm)) - 1;
        const int v = __builtin_amdgcn_readlane(rec_index(lr), k);
        const int j = ref_point(v);
        const int ak = __builtin_amdgcn_readlane(anc, k);
        const float px = readlane_f(lr.x, k), py = readlane_f(lr.y, k), pz = readlane_f(lr.z, k);
        if (v >= 0) {
          if (__builtin_amdgcn_readlane(static_cast<int>(cj), k)) {
            if (ak == root || known_same_set(labels, j, root)) continue;
            if (cell_reaches_point<D>(a.xs, a.n, sa, na, px, py, pz, eps2)) {
              int nr = 0;
              if (lane == 0) nr = uf_union(labels, root, j, a.info);
              root = __shfl(nr, 0);
            }
          } else if (FIRST) {
            if (ak != j || labels[j] != j) continue;  // claimed already (claims are final)
            if (cell_reaches_point<D>(a.xs, a.n, sa, na, px, py, pz, eps2) && lane == 0) uf_claim(labels, j, sa);
          }
          continue;
        }
        if (ak == root || known_same_set(labels, j, root)) continue;
        const float4 blo = make_float4(px, py, pz, 0.0f);
        const float4 bhi = make_float4(readlane_f(hr.x, k), readlane_f(hr.y, k), readlane_f(hr.z, k), 0.0f);
        if (cells_touch<D>(a.xs, a.n, sa, na, j, -a.prim_cnt[__builtin_amdgcn_readlane(r, k)], blo, bhi, eps2)) {
          int nr = 0;
          if (lane == 0) nr = uf_union(labels, root, j, a.info);
          root = __shfl(nr, 0);
        }
      }
      return false;
    });
  }
}

// Main phase, dense cells, when they are many (e.g. a batch of many clouds;
// see cells_lane_mode): one lane per dense cell A, walking (in
// lock-step with the other lanes of its wavefront) with A's box over the
// primitives above A, with the same rules as above; each pair test runs on the
// whole wavefront (64 points per ballot), one pending lane after another.
template <int D, bool ALL_CORE, bool FIRST, bool B>
__global__ void k_main_dbx_cells_lane(TravArgs a) {
  const int nd = *a.d_ndense;
  if (!cells_lane_mode(a)) return;
  const int m = tree_m(a.t);
  const int lane = lane_id();
  const int64_t k = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, nd);
  const bool mine = k >= 0 && k < nd;
  const int A = mine ? a.dense_list[k] : 0;
  const int sa = mine ? a.prim_start[A] : 0;
  const int na = mine ? -a.prim_cnt[A] : 0;
  const Scope sc = scope_of<B>(a, m, sa);
  BoxQ qa;
  {
    const float4 lo = mine ? a.prim_lo[A] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 hi = mine ? a.prim_hi[A] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    qa.lo[0] = lo.x; qa.lo[1] = lo.y; qa.lo[2] = lo.z;
    qa.hi[0] = hi.x; qa.hi[1] = hi.y; qa.hi[2] = hi.z;
  }
  int* labels = a.labels;
  int root = sa;
  Walk w;
  walk_init<true>(w, m, sc, A, mine);
  bool active = mine && !walk_done(w);
  while (ballot(active)) {
    int pend = -1;
    if (active) {
      const int r = walk_step<D, true>(w, a.t, m, qa, sc.eps2, A, a.info);
      if (r >= 0) {
        const float4 lr = a.prim_lo[r];
        const int s = ref_point(rec_index(lr));
        if (rec_index(lr) >= 0) {
          const float px = lr.x, py = lr.y, pz = lr.z;
          if (box_dist2<D>(px, py, pz, qa.lo[0], qa.lo[1], qa.lo[2], qa.hi[0], qa.hi[1], qa.hi[2]) <= sc.eps2) {
            if (ALL_CORE || a.core[s]) {
              if (!known_same_set(labels, s, root)) pend = r;
            } else if (FIRST && labels[s] == s) {
              pend = r;
            }
          }
        } else {
          const float4 blo = lr, bhi = a.prim_hi[r];
          if (boxbox_dist2<D>(qa.lo, qa.hi, blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z) <= sc.eps2 &&
              !known_same_set(labels, s, root))
            pend = r;
        }
      }
    }
    for (uint64_t pm = ballot(pend >= 0); pm; pm &= pm - 1) {
      const int L = __ffsll(static_cast<unsigned long long>(pm)) - 1;
      const int r = __shfl(pend, L);
      const int sA = __shfl(sa, L), nA = __shfl(na, L);
      const float e2 = readlane_f(sc.eps2, L);
      const int c = a.prim_cnt[r], s = a.prim_start[r];
      bool hit;
      if (c > 0) {
        const float px = a.xs[s], py = a.xs[a.n + s], pz = D == 3 ? a.xs[2 * a.n + s] : 0.0f;
        hit = cell_reaches_point<D>(a.xs, a.n, sA, nA, px, py, pz, e2);
      } else {
        hit = cells_touch<D>(a.xs, a.n, sA, nA, s, -c, a.prim_lo[r], a.prim_hi[r], e2);
      }
      if (lane == L && hit) {
        if (c > 0 && !(ALL_CORE || a.core[s]))
          uf_claim(labels, s, sA);  // first-claim mode: a non-core neighbour joins A's cluster
        else
          root = uf_union(labels, root, s, a.info);
      }
    }
    if (active && walk_done(w)) active = false;
  }
}

// Canonical border pass for non-core points (all outside dense cells).
// Queries: the listed non-core points whose neighbours were not all recorded
// by the core pass (which wrote -1 for lone points; the records cover the rest).
template <int D, bool B>
__global__ void k_border_dbx(TravArgs a) {
  const int m = tree_m(a.t);
  const int lane = lane_id();
  const int nq = *a.qborder_n;
  const int64_t k = xcd_spread(blockIdx.x, blockDim.x, threadIdx.x, nq);
  const bool mine = k >= 0 && k < nq;
  const int p = mine ? a.qborder[k] : 0;
  const float4 own = mine ? a.prim_lo[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const int i = mine ? rec_index(own) : 0;
  const Scope sc = scope_of<B>(a, m, i);
  const Query q{own.x, own.y, own.z};
  int best = 0x7fffffff;
  Walk w;
  walk_init<false>(w, m, sc, 0, mine);
  bool active = mine && !walk_done(w);
  while (ballot(active)) {
    int pend = -1;
    if (active) {
      const int r = walk_step<D, false>(w, a.t, m, q, sc.eps2, 0, a.info);
      if (r >= 0) {
        const float4 lr = a.prim_lo[r];
        const int s = rec_index(lr);
        if (s >= 0) {
          if (rec_point_near<D>(lr, q, sc.eps2) && a.core[s]) {
            const int id = a.cid[a.labels[s]];
            best = id < best ? id : best;
          }
        } else if (cell_box_near<D>(a, r, lr, q, sc.eps2) && a.cid[a.labels[ref_point(s)]] < best) {
          pend = r;
        }
      }
    }
    for (uint64_t pm = ballot(pend >= 0); pm; pm &= pm - 1) {
      const int L = __ffsll(static_cast<unsigned long long>(pm)) - 1;
      const int r = __shfl(pend, L);
      const int s = a.prim_start[r];
      const bool hit = cell_reaches_point<D>(a.xs, a.n, s, -a.prim_cnt[r], __shfl(q.x, L), __shfl(q.y, L),
                                             __shfl(q.z, L), readlane_f(sc.eps2, L));
      if (lane == L && hit) {
        const int id = a.cid[a.labels[s]];
        best = id < best ? id : best;
      }
    }
    if (active && (best == 0 || walk_done(w))) active = false;
  }
  if (mine) a.border[i] = best == 0x7fffffff ? -1 : best;
}

// Test hook: one lane walks the tree with an always-true box test and records,
// in order, the leaves a walk masked at `mask` reaches (mask = -1: unmasked).
__global__ void k_debug_walk(TreeView t, int m, int mask, int* out_leaves, int* out_count, int cap,
                             uint32_t* info) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const Query q{0.0f, 0.0f, 0.0f};
  const Scope sc{m == 1 ? kLeaf : 0u, m - 1, INFINITY, 0};
  int cnt = 0;
  traverse<3, true>(t, m, sc, q, mask, info, [&](int l) {
    if (cnt < cap) out_leaves[cnt] = l;
    ++cnt;
    return false;
  });
  *out_count = cnt;
}

// Kernels indexed with xcd_spread(): every XCD needs ceil(ceil(n/8)/block)
// workgroups of its own, so the grid is 8 times that.
inline dim3 grid_of(int64_t n, int block) {
  return dim3(static_cast<unsigned>(kNumXcd * ceil_div(ceil_div(n, kNumXcd), block)));
}

template <int D>
void lone_t(const TravArgs& a, const uint64_t* pkey, const GridPlan* plan, uint32_t* table, uint64_t* words,
            const uint32_t* bounds, int* list, int* list_n, hipStream_t s) {
  // the plan allows a table of at most n / 2 64-bit words (it lives in an n-int buffer)
  const int64_t gc = std::min<int64_t>(std::max<int64_t>(ceil_div(a.n / 2, 256 * 4), 1), 2048);
  hipLaunchKernelGGL(k_lone_clear, dim3(static_cast<unsigned>(gc)), dim3(256), 0, s, plan,
                     reinterpret_cast<uint64_t*>(table));
  const int64_t gb = std::min<int64_t>(ceil_div(a.t.m_cap, 256), 4096);  // 4 wavefronts of 64 primitives
  hipLaunchKernelGGL(k_lone_bits<D>, dim3(static_cast<unsigned>(gb > 0 ? gb : 1)), dim3(256), 0, s, pkey, a.t.d_m,
                     plan, words, table, list_n);
  const int64_t gf = ceil_div(a.t.m_cap, kLoneRounds * 256);
  hipLaunchKernelGGL(k_lone_filter<D>, dim3(static_cast<unsigned>(gf > 0 ? gf : 1)), dim3(256), 0, s, a, pkey, plan,
                     words, table, bounds, list, list_n);
}

template <int D, bool B>
void core_t(const TravArgs& a, bool densebox, hipStream_t s) {
  const dim3 g = grid_of(a.n, a.block), b(a.block);
  const size_t lds = sizeof(int) * kRecNb * a.block;  // neighbour records
  if (densebox && a.core_list) {
    // kNumXcd segments of at most lone_segment(m) <= this many listed queries, or
    // (when the plan turns the list off) every primitive
    const int64_t share = kLoneRounds * 256;
    const int64_t seg = ceil_div(ceil_div(a.t.m_cap, kNumXcd), share) * share;
    const int64_t gl = std::max<int64_t>(kNumXcd * ceil_div(seg, a.block), grid_of(ceil_div(a.n, kCoreQ), a.block).x);
    hipLaunchKernelGGL((k_core_dbx<D, B>), dim3(static_cast<unsigned>(gl)), b, kCoreQ * lds, s, a);
  } else if (densebox) {
    hipLaunchKernelGGL((k_core_dbx<D, B>), grid_of(ceil_div(a.n, kCoreQ), a.block), b, kCoreQ * lds, s, a);
  } else {
    hipLaunchKernelGGL((k_core_fdb<D, B>), g, b, lds, s, a);
  }
}

// part: 0 = everything, 1 = dense-cell queries only, 2 = point queries only (DenseBox)
template <int D, bool ALL, bool FIRST, bool B>
void main_t(const TravArgs& a, bool densebox, int part, hipStream_t s) {
  const dim3 g = grid_of(a.n, a.block), b(a.block);
  if (densebox) {
    if (part != 2) {
      // a batch's many cells usually go to the lane kernel, where this one exits at once
      hipLaunchKernelGGL((k_main_dbx_cells_wave<D, ALL, FIRST, B>), dim3(B ? 2048 : 4096), dim3(256), 0, s, a);
      // dense cells hold >= minPts points each, so there are at most n / minPts
      const int64_t max_cells = a.min_pts > 1 ? a.n / a.min_pts + 1 : a.n;
      if (max_cells > kCellsPerWaveMax)
        hipLaunchKernelGGL((k_main_dbx_cells_lane<D, ALL, FIRST, B>), grid_of(max_cells, a.block), b, 0, s, a);
    }
    if (part != 1)
      hipLaunchKernelGGL((k_main_dbx_points<D, ALL, FIRST, B>), g, b, sizeof(uint32_t) * kWideStack * (a.block / 64), s,
                         a);
  } else if (FIRST) {
    hipLaunchKernelGGL((k_main_fdb_first<D, B>), g, b, 0, s, a);
  } else {
    constexpr int kQ = 1;
    const dim3 gq(static_cast<unsigned>(kNumXcd * ceil_div(ceil_div(a.n, kNumXcd), 256 * kQ)));
    hipLaunchKernelGGL((k_main_fdb_q<D, ALL, B, kQ>), gq, dim3(256), 0, s, a);
  }
}

template <int D, bool B>
void border_t(const TravArgs& a, bool densebox, hipStream_t s) {
  const dim3 g = grid_of(a.n, a.block), b(a.block);
  hipLaunchKernelGGL(k_border_rec, grid_of(a.brec_cap, 256), dim3(256), 0, s, a);
  if (densebox) hipLaunchKernelGGL((k_border_dbx<D, B>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_border_fdb<D, B>), g, b, 0, s, a);
}

template <int D>
void main_dispatch(const TravArgs& a, bool densebox, bool all_core, bool first_border, int part, hipStream_t s) {
  if (a.pkeys != nullptr) {  // batches always run the core pass
    if (first_border) main_t<D, false, true, true>(a, densebox, part, s);
    else main_t<D, false, false, true>(a, densebox, part, s);
  } else if (all_core) {
    main_t<D, true, false, false>(a, densebox, part, s);
  } else if (first_border) {
    main_t<D, false, true, false>(a, densebox, part, s);
  } else {
    main_t<D, false, false, false>(a, densebox, part, s);
  }
}

}  // namespace

void launch_lone_filter(const TravArgs& a, int dim, const uint64_t* prim_key, const GridPlan* plan, uint32_t* table,
                        uint64_t* words, const uint32_t* bounds, int* list, int* list_n, hipStream_t s) {
  if (a.n <= 0) return;
  if (dim == 3) lone_t<3>(a, prim_key, plan, table, words, bounds, list, list_n, s);
  else lone_t<2>(a, prim_key, plan, table, words, bounds, list, list_n, s);
}

void launch_fdb_local(const TravArgs& a, int dim, bool all_core, hipStream_t s) {
  if (a.n <= 1) return;
  const dim3 g(static_cast<unsigned>(ceil_div(a.n, 256))), b(256);
  if (dim == 3) {
    if (all_core) hipLaunchKernelGGL((k_fdb_local<3, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_fdb_local<3, false>), g, b, 0, s, a);
  } else {
    if (all_core) hipLaunchKernelGGL((k_fdb_local<2, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_fdb_local<2, false>), g, b, 0, s, a);
  }
}

void launch_cut_summary(const TravArgs& a, bool all_core, int* sum, hipStream_t s) {
  if (a.n <= 1 || !a.t.cut || !a.t.cut_n) return;
  const int m = static_cast<int>(a.n);
  if (all_core) hipLaunchKernelGGL(k_cut_summary<true>, dim3(kCutMax), dim3(256), 0, s, a.t, m, a.labels, a.core, sum);
  else hipLaunchKernelGGL(k_cut_summary<false>, dim3(kCutMax), dim3(256), 0, s, a.t, m, a.labels, a.core, sum);
}

void launch_core(const TravArgs& a, int dim, bool densebox, hipStream_t s) {
  if (a.n <= 0) return;
  const bool B = a.pkeys != nullptr;
  if (dim == 3) {
    if (B) core_t<3, true>(a, densebox, s);
    else core_t<3, false>(a, densebox, s);
  } else {
    if (B) core_t<2, true>(a, densebox, s);
    else core_t<2, false>(a, densebox, s);
  }
}

void launch_main(const TravArgs& a, int dim, bool densebox, bool all_core, bool first_border, int part,
                 hipStream_t s) {
  if (a.n <= 0) return;
  if (dim == 3) main_dispatch<3>(a, densebox, all_core, first_border, part, s);
  else main_dispatch<2>(a, densebox, all_core, first_border, part, s);
}

void launch_debug_walk(const TreeView& t, int m, int mask, int* out_leaves, int* out_count, int cap,
                       uint32_t* info, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_walk, dim3(1), dim3(64), 0, s, t, m, mask, out_leaves, out_count, cap, info);
}

void launch_border(const TravArgs& a, int dim, bool densebox, hipStream_t s) {
  if (a.n <= 0) return;
  const bool B = a.pkeys != nullptr;
  if (dim == 3) {
    if (B) border_t<3, true>(a, densebox, s);
    else border_t<3, false>(a, densebox, s);
  } else {
    if (B) border_t<2, true>(a, densebox, s);
    else border_t<2, false>(a, densebox, s);
  }
}

}  // namespace fdb
