// Finalisation (Section 4.3: point every label straight at its representative)
// and the output encoding, which the paper leaves open: canonical cluster ids
// 0..K-1 in increasing order of the smallest input index among each cluster's
// core points, -1 for noise, scattered back to input order. Also the device-wide
// exclusive scan used here and by DenseBox.
#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n) {
  int64_t g = ceil_div(n, kBlock * 4);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

__global__ __launch_bounds__(kBlock) void k_iota(int* __restrict__ labels, int64_t n, int* __restrict__ ends,
                                                 int* __restrict__ minorig) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    labels[i] = static_cast<int>(i);
    if (ends) ends[i] = -1;
    if (minorig) minorig[i] = 0x7fffffff;
  }
}

// No unions run now, so roots are fixed; a stale read is an ancestor and the
// walk still ends at the root.
__global__ __launch_bounds__(kBlock) void k_finalize(int* labels, int64_t n, uint32_t* __restrict__ info) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    int r = labels[i];
    for (int64_t it = 0;; ++it) {
      if (r < 0 || r >= n || it > n) {
        atomicOr(info, kInternalBit);
        r = static_cast<int>(i);
        break;
      }
      int p = labels[r];
      if (p == r) break;
      r = p;
    }
    labels[i] = r;
  }
}

// Finalisation fused with the smallest input index per cluster (for when the
// core flags are final): lanes run the same trip count, so a wavefront whose core
// lanes all reach one root reduces first and issues a single atomic.
__global__ __launch_bounds__(kBlock) void k_finalize_min(int* labels, const uint8_t* __restrict__ core,
                                                         const uint32_t* __restrict__ perm, int64_t n,
                                                         int* __restrict__ minorig, uint32_t* __restrict__ bits,
                                                         uint32_t* __restrict__ info) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t base = blockIdx.x * int64_t(kBlock) + (threadIdx.x & ~63); base < n; base += stride) {
    const int64_t i = base + lane;
    if (bits && i < n && (i & 31) == 0) bits[i >> 5] = 0u;  // the leader words, set after this pass
    int r = -1;
    bool valid = false;
    int o = 0x7fffffff;
    if (i < n) {
      r = labels[i];
      valid = core[i] != 0;
      if (valid) o = static_cast<int>(perm[i]);
      for (int64_t it = 0;; ++it) {
        if (r < 0 || r >= n || it > n) {
          atomicOr(info, kInternalBit);
          r = static_cast<int>(i);
          break;
        }
        const int q = labels[r];
        if (q == r) break;
        r = q;
      }
      labels[i] = r;
    }
    const uint64_t vm = ballot(valid);
    if (vm == 0) continue;
    const int leader = __ffsll(static_cast<unsigned long long>(vm)) - 1;
    const int r0 = __shfl(r, leader);
    if (ballot(valid && r != r0) == 0) {
      for (int off = 32; off > 0; off >>= 1) {
        const int y = __shfl_xor(o, off);
        o = y < o ? y : o;
      }
      if (lane == leader) atomicMin(minorig + r0, o);
    } else if (valid) {
      atomicMin(minorig + r, o);
    }
  }
}

// Debug check of the union-find forest the fused main phase leaves (before
// finalisation). Unions hook the larger root under the smaller one and finds only
// shorten paths, so a core point's parent is a core point with a smaller index;
// a claim points a non-core point at a core tree, so any other point's parent is
// itself or a core point. core == nullptr: every point counts as core (minPts <= 2,
// whose flags are set only afterwards). Counts the points that break this in
// *bad and raises kForestBit.
__global__ __launch_bounds__(kBlock) void k_check_forest(const int* __restrict__ labels,
                                                         const uint8_t* __restrict__ core, int64_t n,
                                                         uint32_t* __restrict__ bad, uint32_t* __restrict__ info) {
  uint32_t cnt = 0;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const int p = labels[i];
    bool ok = p >= 0 && p < n;
    if (ok && p != i) {
      const bool ci = core ? core[i] != 0 : true;
      const bool cp = core ? core[p] != 0 : true;
      ok = cp && (!ci || p < i);
    }
    cnt += ok ? 0u : 1u;
  }
  if (cnt) {
    atomicAdd(bad, cnt);
    atomicOr(info, kForestBit);
  }
}

// minPts <= 2 skips the core pass (Algorithm 3). Then every pair within eps is
// a core pair: with minPts = 2 a point is core iff its set has another member,
// with minPts = 1 every point is core.
__global__ __launch_bounds__(kBlock) void k_core_from_sets(const int* __restrict__ labels,
                                                           uint8_t* __restrict__ core, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    int r = labels[i];
    if (r != i) {
      core[i] = 1;
      core[r] = 1;
    }
  }
}

// Smallest input index per cluster. Sorted neighbours mostly share a root, so a
// wavefront whose core lanes all have one root reduces first and issues a
// single atomic instead of 64 on the same word.
__global__ __launch_bounds__(kBlock) void k_minorig(const int* __restrict__ labels, const uint8_t* __restrict__ core,
                                                    const uint32_t* __restrict__ perm, int64_t n,
                                                    int* __restrict__ minorig) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t base = blockIdx.x * int64_t(kBlock) + (threadIdx.x & ~63); base < n; base += stride) {
    const int64_t i = base + lane;
    const bool valid = i < n && core[i];
    const int r = valid ? labels[i] : -1;
    int o = valid ? static_cast<int>(perm[i]) : 0x7fffffff;
    const uint64_t vm = ballot(valid);
    if (vm == 0) continue;
    const int leader = __ffsll(static_cast<unsigned long long>(vm)) - 1;
    const int r0 = __shfl(r, leader);
    if (ballot(valid && r != r0) == 0) {
      for (int off = 32; off > 0; off >>= 1) {
        int y = __shfl_xor(o, off);
        o = y < o ? y : o;
      }
      if (lane == leader) atomicMin(minorig + r0, o);
    } else if (valid) {
      atomicMin(minorig + r, o);
    }
  }
}

// Leader bit of each cluster: the smallest input index among its core points
// (one atomic per cluster, at its root). A cluster's id is the number of
// leaders at smaller input indices.
__global__ __launch_bounds__(kBlock) void k_leader_bits(const int* __restrict__ labels,
                                                        const uint8_t* __restrict__ core,
                                                        const int* __restrict__ minorig, int64_t n,
                                                        uint32_t* __restrict__ bits) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    if (!(core[i] && labels[i] == i)) continue;
    const int o = minorig[i];
    if (o >= 0 && o < n) atomicOr(bits + (o >> 5), 1u << (o & 31));
  }
}

__global__ __launch_bounds__(kBlock) void k_word_popc(const uint32_t* __restrict__ bits, int64_t words,
                                                      int* __restrict__ cnt) {
  for (int64_t w = blockIdx.x * int64_t(kBlock) + threadIdx.x; w < words; w += int64_t(gridDim.x) * kBlock)
    cnt[w] = __popc(bits[w]);
}

__global__ __launch_bounds__(kBlock) void k_cluster_ids(const int* __restrict__ labels,
                                                        const uint8_t* __restrict__ core,
                                                        const int* __restrict__ minorig,
                                                        const uint32_t* __restrict__ bits, const int* __restrict__ wpre,
                                                        int64_t n, const int* __restrict__ total, int* __restrict__ cid) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    if (core[i] && labels[i] == i) cid[i] = leaders_before(bits, wpre, minorig[i], n, total);
}

// Output scatter from sorted order to input order. The destinations are
// random, so every store costs a memory transaction of its own: with PACK the
// core flag rides in bit 30 of the label (cluster ids stay below 2^30), one
// random store per point, and k_split_core unpacks it in a coalesced pass.
constexpr int kCoreBit = 1 << 30;
constexpr int kScatterItems = 4;

template <bool PACK>
__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ labels, const uint8_t* __restrict__ core,
                                                    const uint32_t* __restrict__ perm, const int* __restrict__ cid,
                                                    const int* __restrict__ border, int mode, int64_t n,
                                                    int32_t* __restrict__ out, uint32_t* __restrict__ info) {
  // mode 0: non-core = noise; 1: non-core from the border pass; 2: first claim.
  // kScatterItems points per thread, their loads issued before any store.
  const int64_t stride = int64_t(gridDim.x) * kBlock * kScatterItems;
  for (int64_t base = blockIdx.x * int64_t(kBlock) * kScatterItems + threadIdx.x; base < n; base += stride) {
    uint32_t o[kScatterItems];
    int lab[kScatterItems];
    bool c[kScatterItems];
#pragma unroll
    for (int t = 0; t < kScatterItems; ++t) {
      const int64_t i = base + t * kBlock;
      const bool in = i < n;
      o[t] = in ? perm[i] : 0u;
      c[t] = in && core[i];
      lab[t] = in ? labels[i] : 0;
    }
    int v[kScatterItems];
#pragma unroll
    for (int t = 0; t < kScatterItems; ++t) {
      const int64_t i = base + t * kBlock;
      if (c[t]) v[t] = cid[lab[t]];
      else if (mode == 1) v[t] = i < n ? border[i] : -1;
      else if (mode == 2) v[t] = lab[t] != i ? cid[lab[t]] : -1;
      else v[t] = -1;
    }
#pragma unroll
    for (int t = 0; t < kScatterItems; ++t) {
      const int64_t i = base + t * kBlock;
      if (i >= n) continue;
      if (o[t] >= n) {
        atomicOr(info, kInternalBit);
        continue;
      }
      out[o[t]] = PACK && c[t] && v[t] >= 0 ? (v[t] | kCoreBit) : v[t];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_split_core(int32_t* __restrict__ out, uint8_t* __restrict__ out_core,
                                                       int64_t n) {
  for (int64_t j = blockIdx.x * int64_t(kBlock) + threadIdx.x; j < n; j += int64_t(gridDim.x) * kBlock) {
    const int v = out[j];
    const bool c = v >= 0 && (v & kCoreBit);
    if (c) out[j] = v & ~kCoreBit;
    out_core[j] = c ? 1 : 0;
  }
}

// ---- device-wide exclusive scan of int32 (reduce, scan block sums, apply) ----

__device__ __forceinline__ int wave_inclusive(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ int block_reduce(int x, int* s_w) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  int t = 0;
  for (int j = 0; j < kBlock / 64; ++j) t += s_w[j];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int* __restrict__ in, int64_t n_cap,
                                                        const int* __restrict__ d_n, int* __restrict__ bsums) {
  __shared__ int s_w[kBlock / 64];
  const int64_t n = d_n ? *d_n : n_cap;
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  int x = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n) x += in[i];
  }
  int t = block_reduce(x, s_w);
  if (threadIdx.x == 0) bsums[blockIdx.x] = t;
}

// Exclusive scan of the block sums in place, by one workgroup of kBsumsBlock
// threads: thread t sums its own run of consecutive entries, the run totals are
// scanned across the workgroup, and each thread rescans its run (a few entries
// per thread for the sizes here, so the kernel is two short passes).
constexpr int kBsumsBlock = 1024;

__global__ __launch_bounds__(kBsumsBlock) void k_scan_bsums(int* __restrict__ bsums, int64_t blocks,
                                                            int* __restrict__ d_total, int* __restrict__ bsums2,
                                                            int* __restrict__ d_total2) {
  __shared__ int s_w[kBsumsBlock / 64];
  if (blockIdx.x == 1) {  // a second array, scanned by the second workgroup
    bsums = bsums2;
    d_total = d_total2;
  }
  const int64_t per = (blocks + kBsumsBlock - 1) / kBsumsBlock;
  const int64_t b0 = threadIdx.x * per, b1 = b0 + per < blocks ? b0 + per : blocks;
  int sum = 0;
  for (int64_t i = b0; i < b1; ++i) sum += bsums[i];
  const int inc = wave_inclusive(sum);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) s_w[w] = inc;
  __syncthreads();
  int add = 0;
  for (int j = 0; j < w; ++j) add += s_w[j];
  int run = inc - sum + add;  // exclusive prefix of this thread's run
  for (int64_t i = b0; i < b1; ++i) {
    const int v = bsums[i];
    bsums[i] = run;
    run += v;
  }
  if (threadIdx.x == kBsumsBlock - 1 && d_total) *d_total = run;
}

// Tile position p lives at LDS word p + p/16: thread t's blocked items
// [16t, 16t+16) then sit at 17t + k, so a blocked access hits distinct banks,
// and global memory is read and written striped (coalesced).
__device__ __forceinline__ int scan_lds(int p) { return p + (p >> 4); }

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int* __restrict__ in, int* __restrict__ out, int64_t n_cap,
                                                       const int* __restrict__ d_n, const int* __restrict__ bsums) {
  static_assert(kScanItems == 16, "the LDS padding assumes 16 items per thread");
  __shared__ int s_v[kScanTile + kScanTile / 16];
  __shared__ int s_w[kBlock / 64];
  __shared__ int s_carry;
  const int64_t n = d_n ? *d_n : n_cap;
  const int64_t base = blockIdx.x * int64_t(kScanTile);
  const int tid = threadIdx.x;
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i = base + p;
    s_v[scan_lds(p)] = i < n ? in[i] : 0;
  }
  if (tid == 0) s_carry = bsums[blockIdx.x];
  __syncthreads();
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = s_v[tid * 17 + k];
    sum += v[k];
  }
  const int inc = wave_inclusive(sum);
  const int w = tid >> 6;
  if ((tid & 63) == 63) s_w[w] = inc;
  __syncthreads();
  int run = s_carry + inc - sum;
  for (int j = 0; j < w; ++j) run += s_w[j];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    s_v[tid * 17 + k] = run;
    run += v[k];
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    const int p = k * kBlock + tid;
    const int64_t i = base + p;
    if (i < n) out[i] = s_v[scan_lds(p)];
  }
}

}  // namespace

void device_scan(const int* in, int* out, int64_t n, const int* d_n, int* bsums, int64_t blocks, int* d_total,
                 hipStream_t s) {
  if (n <= 0) {
    if (d_total) fill_u32(reinterpret_cast<uint32_t*>(d_total), 0, 1, s);
    return;
  }
  const int64_t nb = ceil_div(n, kScanTile);
  (void)blocks;
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, in, n, d_n, bsums);
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kBsumsBlock), 0, s, bsums, nb, d_total, nullptr, nullptr);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, in, out, n, d_n, bsums);
}

void scan_block_sums(int* bsums, int64_t blocks, int* d_total, hipStream_t s, int* bsums2, int* d_total2) {
  hipLaunchKernelGGL(k_scan_bsums, dim3(bsums2 ? 2 : 1), dim3(kBsumsBlock), 0, s, bsums, blocks, d_total, bsums2,
                     d_total2);
}

void launch_init_labels(int* labels, int64_t n, hipStream_t s, int* ends, int* minorig) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, n, ends, minorig);
}

void launch_finalize(int* labels, int64_t n, uint32_t* info, hipStream_t s, const uint8_t* core, const uint32_t* perm,
                     int* minorig, uint32_t* bits, bool minorig_init) {
  if (minorig) {
    if (minorig_init) fill_u32(reinterpret_cast<uint32_t*>(minorig), 0x7fffffffu, n, s);
    hipLaunchKernelGGL(k_finalize_min, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, perm, n, minorig, bits,
                       info);
  } else {
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, n, info);
  }
}

void launch_check_forest(const int* labels, const uint8_t* core, int64_t n, uint32_t* bad, uint32_t* info,
                         hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_forest, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, n, bad, info);
}

void launch_core_from_sets(const int* labels, uint8_t* core, int64_t n, int min_pts, hipStream_t s) {
  if (min_pts <= 1) {
    fill_u8(core, 1, n, s);
    return;
  }
  fill_u8(core, 0, n, s);
  hipLaunchKernelGGL(k_core_from_sets, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, n);
}

void canonical_ids(const int* labels, const uint8_t* core, const uint32_t* perm, int64_t n, int* minorig,
                   uint32_t* bits, int* wpre, int* bsums, int64_t scan_blocks, int* cid, int* d_k, hipStream_t s,
                   bool ids, bool minorig_ready) {
  const int g = grid_for(n);
  const int64_t words = ceil_div(n, 32);
  int* cnt = reinterpret_cast<int*>(bits + words);
  if (!minorig_ready) {
    fill_u32(bits, 0, words, s);
    fill_u32(reinterpret_cast<uint32_t*>(minorig), 0x7fffffffu, n, s);
    hipLaunchKernelGGL(k_minorig, dim3(g), dim3(kBlock), 0, s, labels, core, perm, n, minorig);
  }
  hipLaunchKernelGGL(k_leader_bits, dim3(g), dim3(kBlock), 0, s, labels, core, minorig, n, bits);
  hipLaunchKernelGGL(k_word_popc, dim3(grid_for(words)), dim3(kBlock), 0, s, bits, words, cnt);
  device_scan(cnt, wpre, words, nullptr, bsums, scan_blocks, d_k, s);
  if (ids)
    hipLaunchKernelGGL(k_cluster_ids, dim3(g), dim3(kBlock), 0, s, labels, core, minorig, bits, wpre, n, d_k, cid);
}

void launch_scatter(const int* labels, const uint8_t* core, const uint32_t* perm, const int* cid, const int* border,
                    bool first_border, bool have_border, int64_t n, int32_t* out_labels, uint8_t* out_core,
                    uint32_t* info, hipStream_t s) {
  int mode = have_border ? 1 : (first_border ? 2 : 0);
  if (out_core) {
    hipLaunchKernelGGL(k_scatter<true>, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, perm, cid, border,
                       mode, n, out_labels, info);
    hipLaunchKernelGGL(k_split_core, dim3(grid_for(n)), dim3(kBlock), 0, s, out_labels, out_core, n);
  } else {
    hipLaunchKernelGGL(k_scatter<false>, dim3(grid_for(n)), dim3(kBlock), 0, s, labels, core, perm, cid, border,
                       mode, n, out_labels, info);
  }
}

}  // namespace fdb
