// LSD radix sort of (key, index) pairs, 8-bit digits, stable. Section 4.1 sorts
// queries and primitives along a space-filling curve; Karras' hierarchy needs
// the keys sorted with equal keys left in index order, which a stable LSD sort
// started from the identity permutation gives.
//
// Design (after Merrill & Adinets' "onesweep"): one kernel builds the histograms
// of every pass at once; then in each pass a workgroup ranks a tile (5632 32-bit
// or 6144 64-bit keys) with wavefront ballots and scatters it through LDS, so that
// writes are contiguous per digit. A tile learns its global offsets in one of two
// ways. Look-back: a decoupled look-back over earlier tiles (four status words per
// round trip), tiles numbered in the order workgroups start (an atomic ticket), so
// a tile only waits on tiles already running. Reduce-then-scan (the 32-bit passes
// of the sort planned on the device): a count kernel stores every tile's digit
// counts and a scan turns them into offsets before the pass, which then waits on
// nothing. With ~770 tiles in flight at once on 256 CUs, the look-back's walks over
// earlier tiles' uncached status words cost more than the count kernel's extra
// read of the keys (per-tile clocks: ~10 of a tile's ~24 us went to the look-back).
#include "fdb_device.hpp"
#include "fdb_internal.hpp"

namespace fdb {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRadix = 256;

// Look-back status word: [epoch:30][flag:2][count:32]. flag 1 = this tile's own
// count, flag 2 = inclusive prefix through this tile. epoch = pass + 1 tells a
// word of this pass from one left by an earlier pass.
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint64_t flag, uint32_t count) {
  return (uint64_t(epoch) << 34) | (flag << 32) | count;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift) {
  return static_cast<uint32_t>(key >> shift) & 0xffu;
}

// Histogram of every pass's digit over all keys.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_hist(const K* __restrict__ keys, int64_t n, int passes,
                                                 uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8 * kRadix];
  hist_clear(s_h, passes);
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  // every lane of a wavefront runs the same trip count so ballots see all lanes
  const int64_t base0 = blockIdx.x * int64_t(kBlock) + (threadIdx.x & ~63);
  for (int64_t base = base0; base < n; base += stride) {
    int64_t i = base + (threadIdx.x & 63);
    bool valid = i < n;
    hist_add(valid ? keys[i] : K(0), valid, passes, s_h);
  }
  hist_flush(s_h, passes, hist);
}

// Exclusive scan of each pass's 256 digit counts -> global digit offsets, and in
// digoff[8 * 256 + p] a flag (1) for a pass whose digit is the same for every key.
__global__ __launch_bounds__(kRadix) void k_digit_offsets(const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ digoff) {
  __shared__ uint32_t s[kRadix];
  __shared__ uint32_t s_one;
  const int p = blockIdx.x, d = threadIdx.x;
  s[d] = hist[p * kRadix + d];
  if (d == 0) s_one = 0;
  __syncthreads();
  uint32_t tot = 0;
  for (int k = 0; k < kRadix; ++k) tot += s[k];  // every thread, from LDS
  if (tot > 0 && s[d] == tot) s_one = 1;
  __syncthreads();
  if (d == 0) digoff[8 * kRadix + p] = s_one;
  for (int off = 1; off < kRadix; off <<= 1) {
    uint32_t v = d >= off ? s[d - off] : 0;
    __syncthreads();
    s[d] += v;
    __syncthreads();
  }
  digoff[p * kRadix + d] = s[d] - hist[p * kRadix + d];
}

// Pass plan of a host-sequenced sort (one thread): constant-digit passes are
// skipped two at a time, so the number of passes run keeps its parity; each pass
// run gets the buffer it reads. digoff[8 * 256 + p] becomes bit 1 = skip, bit 0 =
// source buffer.
__global__ void k_pass_plan(uint32_t* __restrict__ digoff, int passes) {
  uint32_t* f = digoff + 8 * kRadix;
  bool skip[8];
  for (int p = 0; p < 8; ++p) skip[p] = false;
  for (int p = 0; p + 1 < passes; ++p)
    if (f[p] && f[p + 1]) {
      skip[p] = skip[p + 1] = true;
      ++p;
    }
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    f[p] = (skip[p] ? 2u : 0u) | static_cast<uint32_t>(cur);
    if (!skip[p]) cur ^= 1;
  }
}

// Block-wide exclusive scan of one value per thread (kBlock threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wsum[w] = x;
  __syncthreads();
  uint32_t add = 0;
  for (int j = 0; j < w; ++j) add += s_wsum[j];
  __syncthreads();
  return x - v + add;
}

// Does pass p run, and which buffer does it read (`from`; it writes the other)?
// With a plan (a DenseBox grid sized on the device), the pass runs only if the
// plan's key width is K's and p is below its pass count, and `from` follows the
// plan's start buffer. Without one, the pass plan of k_pass_plan decides: a pass
// whose digit is the same for every key is the identity permutation and is
// skipped (in pairs, so the result still ends in the buffer the host expects).
template <typename K>
__device__ __forceinline__ bool pass_source(int p, const GridPlan* plan, const uint32_t* digoff_all, int& from) {
  if (plan) {
    if (plan->key64 != (sizeof(K) == 8 ? 1 : 0) || p >= plan->passes) return false;
    from = (plan->start ^ p) & 1;
    return true;
  }
  const uint32_t f = digoff_all[8 * kRadix + p];
  if (f & 2u) return false;
  from = static_cast<int>(f & 1u);
  return true;
}

// Reduce step of a pass without look-back: every digit's count in every tile,
// digit-major (counts[d * tiles + tile]) for the scan. Tiles are the pass's.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_tile_counts(const K* __restrict__ k0, const K* __restrict__ k1,
                                                        int64_t n, int p, const GridPlan* __restrict__ plan,
                                                        const uint32_t* __restrict__ digoff_all,
                                                        uint32_t* __restrict__ counts, int64_t tiles) {
  int from = 0;
  if (!pass_source<K>(p, plan, digoff_all, from)) return;  // the whole grid leaves
  const K* __restrict__ kin = from ? k1 : k0;
  constexpr int kItems = sort_items<K>();
  constexpr int kTile = 256 * kItems;
  __shared__ uint32_t s_h[kRadix];
  const int tid = threadIdx.x;
  s_h[tid] = 0;
  __syncthreads();
  const int tile = xcd_block(blockIdx.x, gridDim.x);  // the pass's mapping: it re-reads these keys from L2
  const int64_t base = int64_t(tile) * kTile;
  const int shift = 8 * p;
  K key[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t pos = base + k * kBlock + tid;
    key[k] = pos < n ? kin[pos] : K(0);
  }
  // counts only (no ranks): one LDS atomic per wavefront when its lanes share the
  // digit, else one per lane; the ranking pass's eight-ballot digit match made
  // this kernel VALU-bound (24 us a pass on 8M keys)
#pragma unroll
  for (int k = 0; k < kItems; ++k) hist_add(static_cast<K>(key[k] >> shift), base + k * kBlock + tid < n, 1, s_h);
  __syncthreads();
  counts[int64_t(tid) * tiles + tile] = s_h[tid];
}

// Scan step: for digit d (workgroup d), the digit's global offset plus the
// running sum of its counts in earlier tiles, in place: where each tile's keys of
// digit d start in the output.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_tile_scan(uint32_t* __restrict__ counts, int64_t tiles, int p,
                                                      const GridPlan* __restrict__ plan,
                                                      const uint32_t* __restrict__ digoff_all) {
  int from = 0;
  if (!pass_source<K>(p, plan, digoff_all, from)) return;
  constexpr int kPer = 8;
  __shared__ uint32_t s_wsum[kWaves];
  __shared__ uint32_t s_tot;
  const int d = blockIdx.x, tid = threadIdx.x;
  uint32_t* __restrict__ c = counts + int64_t(d) * tiles;
  uint32_t run = digoff_all[p * kRadix + d];
  for (int64_t c0 = 0; c0 < tiles; c0 += kBlock * kPer) {
    uint32_t v[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t i = c0 + int64_t(tid) * kPer + k;
      v[k] = i < tiles ? c[i] : 0u;
      sum += v[k];
    }
    const uint32_t ex = block_exclusive_scan(sum, s_wsum);
    if (tid == kBlock - 1) s_tot = ex + sum;
    uint32_t r = run + ex;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t i = c0 + int64_t(tid) * kPer + k;
      if (i < tiles) c[i] = r;
      r += v[k];
    }
    __syncthreads();
    run += s_tot;
    __syncthreads();
  }
}

// One pass: reads buffer `from` (pass_source) and writes the other. OFFS: the
// tile follows from the workgroup's index and its offsets come from k_tile_scan
// (offs); otherwise from the look-back.
template <typename K, bool OFFS>
__global__ __launch_bounds__(kBlock) void k_onesweep(K* __restrict__ k0, K* __restrict__ k1,
                                                     uint32_t* __restrict__ v0, uint32_t* __restrict__ v1, int64_t n,
                                                     int p, const GridPlan* __restrict__ plan,
                                                     const uint32_t* __restrict__ digoff_all,
                                                     uint32_t* __restrict__ tilectr_all, uint64_t* __restrict__ status,
                                                     const uint32_t* __restrict__ offs, int64_t otiles,
                                                     uint32_t* __restrict__ info) {
  int from = 0;
  if (!pass_source<K>(p, plan, digoff_all, from)) return;  // the whole grid leaves
  const K* __restrict__ kin = from ? k1 : k0;
  K* __restrict__ kout = from ? k0 : k1;
  const uint32_t* __restrict__ vin = from ? v1 : v0;
  uint32_t* __restrict__ vout = from ? v0 : v1;
  const int shift = 8 * p;

  const uint32_t epoch = static_cast<uint32_t>(p + 1);
  const uint32_t* __restrict__ digoff = digoff_all + p * kRadix;
  uint32_t* __restrict__ tilectr = tilectr_all + p;
  constexpr int kItems = sort_items<K>();
  constexpr int kTile = 256 * kItems;
  static_assert(kTile >= kSortTileMin, "the workspace sizes the status words for kSortTileMin");
  constexpr int kWaveTile = 64 * kItems;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wcnt[kWaves][kRadix];  // per-wave digit counts, then per-wave prefixes
  __shared__ uint32_t s_dstart[kRadix];        // tile-local start of each digit
  __shared__ uint32_t s_gbase[kRadix];         // global start of this tile's run of each digit
  __shared__ uint32_t s_wsum[kWaves];
  __shared__ K s_keys[kTile];
  __shared__ uint32_t s_vals[kTile];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t ntiles = (n + kTile - 1) / kTile;
  // Look-back: a workgroup takes tiles by ticket until none is left, so the grid
  // is what is resident at once rather than a workgroup per tile. OFFS: one tile
  // per workgroup.
  for (;;) {
    if (!OFFS && tid == 0) s_tile = atomicAdd(tilectr, 1u);
    for (int i = tid; i < kWaves * kRadix; i += kBlock) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    // OFFS: tiles laid contiguously per XCD (as in k_tile_counts), so the partial
    // output lines where one tile's run of a digit meets the next tile's are
    // completed in one L2 instead of being written to memory from two
    const int64_t tile = OFFS ? int64_t(xcd_block(blockIdx.x, gridDim.x)) : int64_t(s_tile);
    if (tile >= ntiles) break;  // uniform: s_tile is shared
    const int64_t wbase = tile * kTile + int64_t(w) * kWaveTile;

    K key[kItems];
    uint32_t val[kItems];
    uint32_t rank[kItems];
    // the planned sort's first pass starts from the identity permutation (the key
    // kernel writes no values then)
    const bool iota = plan && p == 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      int64_t pos = wbase + k * 64 + lane;
      bool valid = pos < n;
      key[k] = valid ? kin[pos] : K(0);
      val[k] = valid ? (iota ? static_cast<uint32_t>(pos) : vin[pos]) : 0u;
    }
    // Rank within the wavefront: positions run wave-major, then item, then lane,
    // so processing items in order keeps the sort stable.
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      bool valid = wbase + k * 64 + lane < n;
      uint32_t d = digit_of(key[k], shift);
      uint64_t m = match_digit(d, valid);
      int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
      uint32_t before = 0;
      if (valid && lane == leader) {  // leaders of distinct digits touch distinct words
        before = s_wcnt[w][d];
        s_wcnt[w][d] = before + static_cast<uint32_t>(__popcll(m));
      }
      before = __shfl(before, leader < 0 ? 0 : leader);
      rank[k] = before + static_cast<uint32_t>(__popcll(m & lanemask_lt()));
    }
    __syncthreads();

    // Thread d: prefix over wavefronts and tile total of digit d.
    const uint32_t d = tid;
    uint32_t total = 0;
#pragma unroll
    for (int j = 0; j < kWaves; ++j) {
      uint32_t c = s_wcnt[j][d];
      s_wcnt[j][d] = total;
      total += c;
    }
    // Thread d: its tile's global start for digit d.
    if constexpr (OFFS) {
      s_gbase[d] = offs[int64_t(d) * otiles + tile];
    } else {
      uint64_t* st = status + tile * kRadix + d;
      uint32_t excl = 0;
      if (tile == 0) {
        st_agent64(st, pack_status(epoch, kFlagIncl, total));
      } else {
        st_agent64(st, pack_status(epoch, kFlagAgg, total));
        int spins = 0;
        for (int64_t j = tile - 1; j >= 0;) {
          // four predecessors per round trip
          uint64_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = j - u >= 0 ? ld_agent64(status + (j - u) * kRadix + d) : 0;
          bool done = false, wait = false;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (done || wait || j < 0) continue;
            if (static_cast<uint32_t>(v[u] >> 34) != epoch) {
              wait = true;
              continue;
            }
            excl += static_cast<uint32_t>(v[u]);
            if (((v[u] >> 32) & 3u) == kFlagIncl) done = true;
            else --j;
          }
          if (done) break;
          if (wait) {
            if (++spins > (1 << 24)) {
              atomicOr(info, kInternalBit);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        st_agent64(st, pack_status(epoch, kFlagIncl, excl + total));
      }
      s_gbase[d] = digoff[d] + excl;
    }
    uint32_t ds = block_exclusive_scan(total, s_wsum);
    s_dstart[d] = ds;
    __syncthreads();

    // Local scatter into LDS in sorted order.
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (wbase + k * 64 + lane < n) {
        uint32_t dk = digit_of(key[k], shift);
        uint32_t pos = s_dstart[dk] + s_wcnt[w][dk] + rank[k];
        s_keys[pos] = key[k];
        s_vals[pos] = val[k];
      }
    }
    __syncthreads();
    const int64_t tile_n = n - tile * kTile < kTile ? n - tile * kTile : kTile;
    for (int i = tid; i < tile_n; i += kBlock) {
      K kk = s_keys[i];
      uint32_t dk = digit_of(kk, shift);
      uint32_t dest = s_gbase[dk] + (i - s_dstart[dk]);
      if (dest >= n) {  // only after a failed look-back
        atomicOr(info, kInternalBit);
        continue;
      }
      kout[dest] = kk;
      vout[dest] = s_vals[i];
    }
    if (OFFS) break;
    __syncthreads();  // the next tile reuses the LDS
  }
}

// Workgroups of a look-back pass: at most what is resident at once on 256 CUs
// (two 64-bit or three 32-bit tiles per CU, bound by registers); they loop over
// the tiles.
template <typename K>
unsigned lookback_grid(int64_t tiles) {
  const int64_t cap = (sizeof(K) == 8 ? 2 : 3) * 256;
  return static_cast<unsigned>(tiles < cap ? tiles : cap);
}

template <typename K>
int radix_sort_t(K* keys0, K* keys1, uint32_t* vals0, uint32_t* vals1, int64_t n, int bits, uint32_t* hist,
                 bool hist_ready, uint32_t* digoff, uint32_t* tilectr, uint64_t* status, uint32_t* info,
                 hipStream_t s) {
  const int passes = (bits + 7) / 8;
  if (n <= 1 || passes == 0) return 0;
  const int64_t tiles = ceil_div(n, 256 * sort_items<K>());
  fill_u32(tilectr, 0, passes, s);
  fill_u32(reinterpret_cast<uint32_t*>(status), 0, tiles * kRadix * 2, s);
  if (!hist_ready) {
    fill_u32(hist, 0, passes * kRadix, s);
    int hg = static_cast<int>(ceil_div(n, kBlock * 16));
    if (hg > 2048) hg = 2048;
    hipLaunchKernelGGL(k_hist<K>, dim3(hg), dim3(kBlock), 0, s, keys0, n, passes, hist);
  }
  hipLaunchKernelGGL(k_digit_offsets, dim3(passes), dim3(kRadix), 0, s, hist, digoff);
  hipLaunchKernelGGL(k_pass_plan, dim3(1), dim3(1), 0, s, digoff, passes);
  // (look-back passes: for 64-bit keys, a count kernel's second read of the keys
  // and its extra launches cost more than the look-back; measured on the Morton
  // and batch sorts)
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_onesweep<K, false>), dim3(lookback_grid<K>(tiles)), dim3(kBlock), 0, s, keys0, keys1,
                       vals0, vals1, n, p, static_cast<const GridPlan*>(nullptr), digoff, tilectr, status,
                       static_cast<const uint32_t*>(nullptr), int64_t(0), info);
    cur ^= 1;
  }
  return cur;
}

}  // namespace

// Look-back words of the planned sort's 64-bit passes (the 32-bit passes keep
// their tile counts in the same buffer; a call runs one width only).
int64_t planned_status_words(int64_t n) { return ceil_div(n, 256 * sort_items<uint64_t>()) * kRadix * 2; }

void radix_sort_planned(void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, int64_t n, const GridPlan* plan,
                        const uint32_t* hist, uint32_t* digoff, uint32_t* tilectr, uint64_t* status,
                        uint32_t* info, hipStream_t s, bool clear) {
  if (n <= 1) return;  // the key kernel's start buffer already is buffer 1 when there is nothing to sort
  const int64_t tiles32 = ceil_div(n, 256 * sort_items<uint32_t>());
  const int64_t tiles64 = ceil_div(n, 256 * sort_items<uint64_t>());
  if (clear) {
    fill_u32(tilectr, 0, 8, s);
    fill_u32(reinterpret_cast<uint32_t*>(status), 0, planned_status_words(n), s);
  }
  hipLaunchKernelGGL(k_digit_offsets, dim3(8), dim3(kRadix), 0, s, hist, digoff);
  // 32-bit keys (at most 4 passes): reduce, scan, then the pass, the tile counts
  // in the look-back buffer (tiles32 * 256 words of its tiles32 * 512)
  uint32_t* counts = reinterpret_cast<uint32_t*>(status);
  uint32_t* k32[2] = {static_cast<uint32_t*>(keys0), static_cast<uint32_t*>(keys1)};
  for (int p = 0; p < 4; ++p) {
    hipLaunchKernelGGL(k_tile_counts<uint32_t>, dim3(static_cast<unsigned>(tiles32)), dim3(kBlock), 0, s, k32[0],
                       k32[1], n, p, plan, digoff, counts, tiles32);
    hipLaunchKernelGGL(k_tile_scan<uint32_t>, dim3(kRadix), dim3(kBlock), 0, s, counts, tiles32, p, plan, digoff);
    hipLaunchKernelGGL((k_onesweep<uint32_t, true>), dim3(static_cast<unsigned>(tiles32)), dim3(kBlock), 0, s, k32[0],
                       k32[1], vals0, vals1, n, p, plan, digoff, tilectr, status,
                       static_cast<const uint32_t*>(counts), tiles32, info);
  }
  for (int p = 0; p < 8; ++p)  // 64-bit keys
    hipLaunchKernelGGL((k_onesweep<uint64_t, false>), dim3(lookback_grid<uint64_t>(tiles64)), dim3(kBlock), 0, s,
                       static_cast<uint64_t*>(keys0), static_cast<uint64_t*>(keys1), vals0, vals1, n, p, plan,
                       digoff, tilectr, status, static_cast<const uint32_t*>(nullptr), int64_t(0), info);
}

int radix_sort(void* keys0, void* keys1, uint32_t* vals0, uint32_t* vals1, int64_t n, bool key64, int bits,
               uint32_t* hist, bool hist_ready, uint32_t* digoff, uint32_t* tilectr, uint64_t* status,
               uint32_t* info, hipStream_t s) {
  if (key64)
    return radix_sort_t(static_cast<uint64_t*>(keys0), static_cast<uint64_t*>(keys1), vals0, vals1, n, bits, hist,
                        hist_ready, digoff, tilectr, status, info, s);
  return radix_sort_t(static_cast<uint32_t*>(keys0), static_cast<uint32_t*>(keys1), vals0, vals1, n, bits, hist,
                      hist_ready, digoff, tilectr, status, info, s);
}

}  // namespace fdb
