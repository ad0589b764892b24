// C ABI of libfdbscan and the launch sequence of one clustering call.
//
// FDbscan (Section 4.1): bounds -> Morton keys -> radix sort -> gather to SoA ->
// LBVH (Karras hierarchy, ropes, refit) -> core pass if minPts > 2 (early exit
// at minPts) -> fused masked traversal with union-find -> finalisation ->
// canonical ids (and the border pass) -> scatter to input order.
// FDbscan-DenseBox (Section 4.2): bounds (read back once to size the grid) ->
// grid-cell keys -> radix sort -> gather -> dense cells + mixed primitives ->
// LBVH over the primitives -> core pass over points outside dense cells ->
// fused traversal -> the same tail.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fdb_internal.hpp"
#include "fdbscan.h"

namespace fdb {

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Plan make_plan(int64_t n, int dim, int algo, int num_clouds) {
  Plan p;
  p.n = n;
  p.dim = dim;
  p.algo = algo;
  p.num_clouds = num_clouds;
  const size_t N = static_cast<size_t>(n > 0 ? n : 1);
  p.sort_tiles = ceil_div(static_cast<int64_t>(N), kSortTileMin);
  p.scan_blocks = ceil_div(static_cast<int64_t>(N), kScanTile);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p.bounds = take(8 * sizeof(uint32_t));
  p.misc = take(kMiscCount * sizeof(int));
  p.gplan = take(sizeof(GridPlan));
  p.keys0 = take(N * 8);
  p.keys1 = take(N * 8);
  p.vals0 = take(N * 4);
  p.vals1 = take(N * 4);
  p.hist = take(8 * 256 * 4);
  p.digoff = take((8 * 256 + 8) * 4);  // digit offsets of 8 passes, then a "digit constant" flag per pass
  p.tilectr = take(64);
  p.status = take(static_cast<size_t>(p.sort_tiles) * 256 * 8);
  p.xs = take(static_cast<size_t>(dim) * N * 4);
  p.node_a = take(N * 32);  // interleaved node records (kNodeStride float4 per node)
  p.node_b = p.node_a + 16;
  p.rope = take(N * 4);
  p.leaf_rope = take(N * 4);
  p.ends = take(N * 4);
  p.cut = take(static_cast<size_t>(kCutMax) * 36);  // kCutMax box pairs, then a summary word each
  p.other = take(N * 4);
  p.gamma = take(N * 4);
  p.labels = take(N * 4);
  p.core = take(N);
  p.lone = take(N);
  p.qborder = take(N * 4);
  p.brec_cap = std::max<int64_t>(4096, static_cast<int64_t>(N) / 8);
  p.brec_i = take(static_cast<size_t>(p.brec_cap) * 4);
  p.brec_nb = take(static_cast<size_t>(p.brec_cap) * kRecNb * 4);
  p.minorig = take(N * 4);
  p.lflag = take(N * 4);
  p.rank = take(N * 4);
  p.bsums = take(static_cast<size_t>(p.scan_blocks + 1) * 4);
  p.cid = take(N * 4);
  p.border = take(N * 4);
  p.cell_id = p.cell_start = p.cand = p.cell_dense = p.cell_lo = p.cell_hi = 0;
  p.pflag = p.prim_start = p.prim_cnt = p.prim_lo = p.prim_hi = p.prim_key = p.dense_list = 0;
  if (algo != FDB_ALGO_FDBSCAN) {  // DenseBox, or the automatic choice (which starts as DenseBox)
    p.cell_id = take(N * 4);
    p.cell_start = take((N + 1) * 4);
    p.cand = take(N * 4);
    p.cell_dense = take(N);
    p.cell_lo = take(N * 16);
    p.cell_hi = take(N * 16);
    p.pflag = take(N * 4);
    p.prim_start = take(N * 4);
    p.prim_cnt = take(N * 4);
    p.prim_lo = take(N * 16);
    p.prim_hi = take(N * 16);
    p.prim_key = take(N * 8);
    p.dense_list = take(N * 4);
    // the cell boxes are dead once the primitives are written: the isolated-point
    // test keeps its occupancy words there
    p.map_bytes = static_cast<int64_t>(p.cell_hi + N * 16 - p.cell_lo);
  }
  p.cl_lo = p.cl_scale = p.cl_eps2 = p.cl_minpts = p.cl_root = p.cl_end = p.cl_flags = p.cl_ord = 0;
  if (num_clouds > 0) {
    const size_t B = static_cast<size_t>(num_clouds);
    p.cl_lo = take(B * 16);
    p.cl_scale = take(B * 16);
    p.cl_eps2 = take(B * 4);
    p.cl_minpts = take(B * 4);
    p.cl_root = take(B * 4);
    p.cl_end = take(B * 4);
    p.cl_flags = take(B * 4);
    p.cl_ord = take(B * 32);
  }
  p.bytes = off;
  return p;
}

struct StageRec {
  const char* name;
  hipEvent_t a, b;
};

// A recorded launch sequence: the call's arguments (every pointer, size and
// parameter but the stream) and the executable graph replaying it.
struct GraphRec {
  std::vector<uint64_t> key;
  hipGraphExec_t exec;
};

// One autotuner result: the launch shape measured fastest for calls of this class.
struct TuneEntry {
  int32_t batched, algo, dim, nlog2, mpclass;  // the class
  int32_t leaf_size, block_size, tile;         // its shape
  double best_ms, default_ms, dense_share;     // what the tuner measured
};

}  // namespace fdb

struct fdb_handle {
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* d_info = nullptr;
  uint32_t* h_pinned = nullptr;  // 16 words of pinned host memory for read-backs
  uint32_t host_info = 0;
  hipStream_t last_stream = nullptr;
  const int* last_misc = nullptr;  // device counters of the last call (in its workspace)
  bool last_densebox = false;
  int64_t last_n = 0;
  bool timing = false;
  int32_t timed_calls = 0;
  std::vector<fdb::StageRec> pending;  // event pairs of the calls since the last collection
  std::vector<std::string> names;      // accumulated stage names (static strings)
  std::vector<double> ms;
  std::vector<hipEvent_t> event_pool;
  std::atomic<int> busy{0};             // a host thread is inside a call (FDB_ERR_BUSY for another)
  hipStream_t cap_stream = nullptr;     // stream that graph recordings are captured on
  std::vector<fdb::GraphRec> graphs;    // recorded launch sequences, most recent last
  std::vector<fdb::TuneEntry> tune;     // launch shapes chosen by fdb_tune (and the tune cache file)
  void* scratch = nullptr;              // this device's copy of the library's static scratch (device address)
};

// Workspace of fdb_dbscan_noalloc: device memory of the library itself, one copy
// per GPU that the library runs on, held until the process ends. In host code this
// name is a host-side stand-in, never a device address: fdb_create looks up the
// current device's copy with hipGetSymbolAddress (once per device) and every
// launch takes that pointer, as it takes a caller's workspace.
static __device__ __align__(256) unsigned char scratch[FDB_NOALLOC_SCRATCH_BYTES];

namespace {

using fdb::ceil_div;

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// The device address of `scratch` on `device` (the current device), looked up on
// the first request for that device.
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device >= 0 && device < kScratchDevices && g_scratch_ptr[device]) return g_scratch_ptr[device];
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (device >= 0 && device < kScratchDevices) g_scratch_ptr[device] = p;
  return p;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

hipEvent_t take_event(fdb_handle* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Marks the start of a named stage; the previous stage (if any) ends there.
// Off while a launch sequence is recorded into a graph.
struct Stager {
  fdb_handle* h;
  hipStream_t s;
  bool on;
  const char* cur = nullptr;
  hipEvent_t cur_a = nullptr;
  Stager(fdb_handle* hh, hipStream_t ss, bool enable) : h(hh), s(ss), on(enable) {}
  void mark(const char* name) {
    if (!on) return;
    hipEvent_t e = take_event(h);
    if (!e) return;
    (void)hipEventRecord(e, s);
    if (cur) {
      hipEvent_t e2 = take_event(h);
      if (e2) {
        (void)hipEventRecord(e2, s);
        h->pending.push_back({cur, cur_a, e2});
      }
    }
    cur = name;
    cur_a = e;
  }
  void finish() {
    if (!on || !cur) return;
    hipEvent_t e2 = take_event(h);
    if (e2) {
      (void)hipEventRecord(e2, s);
      h->pending.push_back({cur, cur_a, e2});
    }
    cur = nullptr;
  }
};

fdb_status collect_timing(fdb_handle* h) {
  for (auto& r : h->pending) {
    if (hipEventSynchronize(r.b) != hipSuccess) return FDB_ERR_HIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return FDB_ERR_HIP;
    size_t k = 0;
    while (k < h->names.size() && h->names[k] != r.name) ++k;
    if (k == h->names.size()) {
      h->names.emplace_back(r.name);
      h->ms.push_back(0.0);
    }
    h->ms[k] += t;
    h->event_pool.push_back(r.a);
    h->event_pool.push_back(r.b);
  }
  h->pending.clear();
  return FDB_OK;
}

bool valid_options(const fdb_options& o) {
  if (o.algo != FDB_ALGO_FDBSCAN && o.algo != FDB_ALGO_DENSEBOX && o.algo != FDB_ALGO_AUTO) return false;
  if (o.border != FDB_BORDER_CANONICAL && o.border != FDB_BORDER_FIRST && o.border != FDB_BORDER_NONE) return false;
  if (o.leaf_size < 0 || o.leaf_size > 1024) return false;
  if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 1024 || o.block_size % 64 != 0)) return false;
  if (o.tile != 0 && (o.tile < 8 || o.tile > 64)) return false;
  if (o.flags & ~uint32_t(FDB_FLAG_GRAPH | FDB_FLAG_VALIDATE)) return false;
  return true;
}

constexpr int kDefaultLeaf = 8;     // measured against 2, 4, 6 and 16 (8M set and the 4096-cloud batch)
constexpr int kDefaultBlock = 128;  // measured against 64, 256 and 512
constexpr int kDefaultTile = 64;    // packet bucket: a candidate per lane (measured against 32)
constexpr size_t kMaxGraphs = 16;

// One host thread per handle: a second one gets FDB_ERR_BUSY instead of racing.
struct CallGuard {
  fdb_handle* h;
  bool ok;
  explicit CallGuard(fdb_handle* hh) : h(hh) {
    int expected = 0;
    ok = h->busy.compare_exchange_strong(expected, 1);
  }
  ~CallGuard() {
    if (ok) h->busy.store(0);
  }
};

struct SingleArgs {
  const float* points;
  int64_t n;
  int32_t dim;
  float eps;
  int32_t min_pts;
  int32_t* labels;
  uint8_t* is_core;
};

struct BatchArgs {
  const float* points;
  int64_t n_total;
  const int64_t* offsets;
  int32_t num_clouds;
  int32_t dim;
  const float* eps;
  const int32_t* min_pts;
  int32_t* labels;
  uint8_t* is_core;
  int32_t* num_clusters;
};

using CallKey = std::vector<uint64_t>;

uint64_t ptr_word(const void* p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); }

uint64_t float_word(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

void options_words(CallKey& k, const fdb_options& o) {
  k.push_back(uint64_t(uint32_t(o.algo)) | uint64_t(uint32_t(o.border)) << 32);
  k.push_back(uint64_t(uint32_t(o.leaf_size)) | uint64_t(uint32_t(o.block_size)) << 32);
  k.push_back(uint64_t(uint32_t(o.tile)) | uint64_t(o.flags) << 32);
}

CallKey single_key(const SingleArgs& a, const fdb_options& o, const void* ws, size_t ws_bytes) {
  CallKey k{1, ptr_word(a.points), uint64_t(a.n), uint64_t(uint32_t(a.dim)), float_word(a.eps),
            uint64_t(uint32_t(a.min_pts)), ptr_word(a.labels), ptr_word(a.is_core), ptr_word(ws), ws_bytes};
  options_words(k, o);
  return k;
}

CallKey batch_key(const BatchArgs& a, const fdb_options& o, const void* ws, size_t ws_bytes) {
  CallKey k{2, ptr_word(a.points), uint64_t(a.n_total), ptr_word(a.offsets), uint64_t(uint32_t(a.num_clouds)),
            uint64_t(uint32_t(a.dim)), ptr_word(a.eps), ptr_word(a.min_pts), ptr_word(a.labels), ptr_word(a.is_core),
            ptr_word(a.num_clusters), ptr_word(ws), ws_bytes};
  options_words(k, o);
  return k;
}

void drop_graphs(fdb_handle* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

// Replays the graph recorded for `key` on `stream`, recording it first (by stream
// capture of launch(cs) on the handle's capture stream) if there is none.
template <typename F>
fdb_status run_graph(fdb_handle* h, const CallKey& key, hipStream_t stream, F&& launch) {
  size_t k = 0;
  while (k < h->graphs.size() && h->graphs[k].key != key) ++k;
  if (k == h->graphs.size()) {
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      h->cap_stream = nullptr;
      return FDB_ERR_HIP;
    }
    hipStream_t cs = h->cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return FDB_ERR_HIP;
    const fdb_status st = launch(cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (st != FDB_OK || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return st != FDB_OK ? st : FDB_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess || !exec) return FDB_ERR_HIP;
    if (h->graphs.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(h->graphs.front().exec);
      h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({key, exec});
    k = h->graphs.size() - 1;
  }
  return hipGraphLaunch(h->graphs[k].exec, stream) == hipSuccess ? FDB_OK : FDB_ERR_HIP;
}

// The caller's workspace (checked against the plan), or the handle's own, grown
// when needed (which drops the graphs recorded over the old one).
fdb_status take_workspace(fdb_handle* h, const fdb::Plan& plan, void* workspace, size_t workspace_bytes,
                          hipStream_t stream, void** out) {
  if (workspace) {
    if (workspace_bytes < plan.bytes) return FDB_ERR_NOMEM;
    *out = workspace;
    return FDB_OK;
  }
  if (h->ws_bytes < plan.bytes) {
    if (h->ws) {
      if (hipStreamSynchronize(stream) != hipSuccess) return FDB_ERR_HIP;
      if (h->cap_stream && hipStreamSynchronize(h->cap_stream) != hipSuccess) return FDB_ERR_HIP;
      if (hipDeviceSynchronize() != hipSuccess) return FDB_ERR_HIP;  // graphs replayed on other streams
      drop_graphs(h);
      (void)hipFree(h->ws);
      h->ws = nullptr;
      h->ws_bytes = 0;
    }
    if (hipMalloc(&h->ws, plan.bytes) != hipSuccess) return FDB_ERR_NOMEM;
    h->ws_bytes = plan.bytes;
  }
  *out = h->ws;
  return FDB_OK;
}

int nlog2_of(int64_t n) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

int mpclass_of(int32_t min_pts) { return min_pts <= 2 ? 0 : 1; }

const fdb::TuneEntry* find_tune(const fdb_handle* h, int batched, int algo, int dim, int64_t n, int mpclass) {
  const int nl = nlog2_of(n);
  for (const auto& e : h->tune)
    if (e.batched == batched && e.algo == algo && e.dim == dim && e.nlog2 == nl && e.mpclass == mpclass) return &e;
  return nullptr;
}

// Launch-shape fields left at 0 take the tuned value for the call's class.
void resolve_shape(const fdb_handle* h, fdb_options& o, int64_t n, int dim, int num_clouds, int32_t min_pts = 3) {
  if (o.leaf_size && o.block_size && o.tile) return;
  const int algo = o.algo == FDB_ALGO_FDBSCAN ? FDB_ALGO_FDBSCAN : FDB_ALGO_DENSEBOX;
  const fdb::TuneEntry* e = find_tune(h, num_clouds > 0, algo, dim, n, num_clouds > 0 ? 1 : mpclass_of(min_pts));
  if (!e) return;
  if (!o.leaf_size) o.leaf_size = e->leaf_size;
  if (!o.block_size) o.block_size = e->block_size;
  if (!o.tile) o.tile = e->tile;
}

fdb_status dbscan_launch(fdb_handle* h, const SingleArgs& args, const fdb_options& o, const fdb::Plan& plan, void* ws,
                         hipStream_t stream, bool timing);
fdb_status batched_launch(fdb_handle* h, const BatchArgs& args, const fdb_options& o, const fdb::Plan& plan, void* ws,
                          hipStream_t stream, bool timing);
fdb_status dbscan_batched_entry(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                                int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                                const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* num_clusters,
                                void* workspace, size_t workspace_bytes, hipStream_t stream);
void load_tune_file(fdb_handle* h);
fdb_status dbscan_entry(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                        const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                        void* workspace, size_t workspace_bytes, hipStream_t stream, bool may_time = true);

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace

extern "C" {

const char* fdb_status_string(fdb_status s) {
  switch (s) {
    case FDB_OK: return "ok";
    case FDB_ERR_INVALID: return "invalid argument";
    case FDB_ERR_NOMEM: return "workspace too small or allocation failed";
    case FDB_ERR_HIP: return "HIP runtime error";
    case FDB_ERR_NONFINITE: return "non-finite coordinate";
    case FDB_ERR_INTERNAL: return "internal consistency check failed";
    case FDB_ERR_BUSY: return "another thread is inside a call on this handle";
    case FDB_ERR_SCRATCH:
      return "input needs more workspace than the library's static scratch (FDB_NOALLOC_SCRATCH_BYTES)";
  }
  return "unknown status";
}

fdb_status fdb_create(fdb_handle** out, int device) {
  if (!out) return FDB_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return FDB_ERR_HIP;
  if (device < 0 || device >= count) return FDB_ERR_INVALID;
  fdb_handle* h = new (std::nothrow) fdb_handle();
  if (!h) return FDB_ERR_NOMEM;
  h->device = device;
  DeviceGuard g(device);
  if (hipMalloc(&h->d_info, 256) != hipSuccess) {
    delete h;
    return FDB_ERR_NOMEM;
  }
  if (hipHostMalloc(&h->h_pinned, 16 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(h->d_info);
    delete h;
    return FDB_ERR_NOMEM;
  }
  h->scratch = scratch_address(device);  // nullptr: fdb_dbscan_noalloc reports FDB_ERR_HIP
  load_tune_file(h);
  *out = h;
  return FDB_OK;
}

void fdb_destroy(fdb_handle* h) {
  if (!h) return;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  for (auto& r : h->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->ws) (void)hipFree(h->ws);
  if (h->d_info) (void)hipFree(h->d_info);
  if (h->h_pinned) (void)hipHostFree(h->h_pinned);
  delete h;
}

fdb_status fdb_workspace_bytes(int64_t n, int32_t dim, const fdb_options* opt, size_t* h_out) {
  if (!h_out) return FDB_ERR_INVALID;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o) || (dim != 2 && dim != 3) || n < 0 || n > fdb::kMaxPoints) return FDB_ERR_INVALID;
  *h_out = fdb::make_plan(n, dim, o.algo).bytes;
  return FDB_OK;
}

fdb_status fdb_last_status(fdb_handle* h, hipStream_t stream, uint32_t* h_info) {
  if (!h || !h_info) return FDB_ERR_INVALID;
  DeviceGuard g(h->device);
  if (hipMemcpyAsync(h->h_pinned + 8, h->d_info, 4, hipMemcpyDeviceToHost, stream) != hipSuccess)
    return FDB_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return FDB_ERR_HIP;
  *h_info = h->h_pinned[8] | h->host_info;
  if (*h_info & FDB_INFO_NONFINITE) return FDB_ERR_NONFINITE;
  if (*h_info & FDB_INFO_INTERNAL) return FDB_ERR_INTERNAL;
  return FDB_OK;
}

fdb_status fdb_last_info(fdb_handle* h, uint32_t* h_info) {
  if (!h || !h_info) return FDB_ERR_INVALID;
  const fdb_status st = fdb_last_status(h, h->last_stream, h_info);
  return st == FDB_ERR_NONFINITE || st == FDB_ERR_INTERNAL ? FDB_OK : st;
}

fdb_status fdb_last_counts(fdb_handle* h, int64_t* h_counts) {
  if (!h || !h_counts) return FDB_ERR_INVALID;
  for (int k = 0; k < 4; ++k) h_counts[k] = 0;
  if (!h->last_misc) return FDB_OK;
  DeviceGuard g(h->device);
  if (hipMemcpyAsync(h->h_pinned, h->last_misc, 5 * sizeof(int), hipMemcpyDeviceToHost, h->last_stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->last_stream) != hipSuccess)
    return FDB_ERR_HIP;
  const int32_t* v = reinterpret_cast<const int32_t*>(h->h_pinned);
  h_counts[0] = v[fdb::kMiscNumClusters];
  if (h->last_densebox) {
    h_counts[1] = v[fdb::kMiscNumCells];
    h_counts[2] = v[fdb::kMiscNumDense];
    h_counts[3] = v[fdb::kMiscNumPrims];
  } else {
    h_counts[3] = h->last_n;
  }
  return FDB_OK;
}

fdb_status fdb_debug_forest(fdb_handle* h, const int32_t* parent, const uint8_t* is_core, int64_t n,
                            int64_t* h_bad) {
  if (!h || !h_bad || n < 0 || n > fdb::kMaxPoints || (n > 0 && !parent)) return FDB_ERR_INVALID;
  DeviceGuard g(h->device);
  hipStream_t s = nullptr;
  fdb::fill_u32(h->d_info, 0, 2, s);
  fdb::launch_check_forest(parent, is_core, n, h->d_info + 1, h->d_info, s);
  if (hipMemcpy(h->h_pinned, h->d_info, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return FDB_ERR_HIP;
  *h_bad = h->h_pinned[1];
  return FDB_OK;
}

fdb_status fdb_debug_lbvh(fdb_handle* h, const uint64_t* h_keys, int32_t m, int32_t mask, int32_t leaf_size,
                          int32_t* h_gamma, int32_t* h_other, int32_t* h_leaves, int32_t* h_num_leaves) {
  using namespace fdb;
  if (!h || !h_keys || m < 1 || m > (1 << 24) || mask < -1 || mask >= m || leaf_size < 1 || leaf_size > 1024 ||
      !h_leaves || !h_num_leaves || (m > 1 && (!h_gamma || !h_other)))
    return FDB_ERR_INVALID;
  for (int32_t k = 1; k < m; ++k)
    if (h_keys[k] < h_keys[k - 1]) return FDB_ERR_INVALID;
  DeviceGuard g(h->device);
  const size_t M = static_cast<size_t>(m);
  void* buf = nullptr;
  const size_t bytes = M * 8 + 3 * M * 4 + 2 * M * 16 + 2 * M * 4 + 2 * M * 4 + 3 * M * 4 + M * 4 + 256;
  if (hipMalloc(&buf, bytes) != hipSuccess) return FDB_ERR_NOMEM;
  char* p = static_cast<char*>(buf);
  uint64_t* keys = reinterpret_cast<uint64_t*>(p); p += M * 8;
  float* xs = reinterpret_cast<float*>(p); p += 3 * M * 4;
  float4* na = reinterpret_cast<float4*>(p); p += 2 * M * 16;  // interleaved node records
  float4* nb = na + 1;
  int* rope = reinterpret_cast<int*>(p); p += M * 4;
  int* lrope = reinterpret_cast<int*>(p); p += M * 4;
  int* ends = reinterpret_cast<int*>(p); p += M * 4;
  int* other = reinterpret_cast<int*>(p); p += M * 4;
  int* gamma = reinterpret_cast<int*>(p); p += M * 4;
  int* leaves = reinterpret_cast<int*>(p); p += M * 4;
  int* count = reinterpret_cast<int*>(p);
  fdb_status st = FDB_OK;
  hipStream_t s = nullptr;
  if (hipMemcpy(keys, h_keys, M * 8, hipMemcpyHostToDevice) != hipSuccess) st = FDB_ERR_HIP;
  if (st == FDB_OK) {
    fill_u32(reinterpret_cast<uint32_t*>(xs), 0, 3 * M, s);
    fill_u32(h->d_info, 0, 1, s);
    build_lbvh(keys, true, m, 3, xs, m, nullptr, nullptr, na, nb, rope, lrope, ends, other, gamma, nullptr,
               h->d_info, s);
    TreeView t{na, nb, rope, lrope, m, nullptr, leaf_size};
    launch_debug_walk(t, m, mask, leaves, count, m, h->d_info, s);
    if (hipStreamSynchronize(s) != hipSuccess) st = FDB_ERR_HIP;
  }
  if (st == FDB_OK && m > 1 &&
      (hipMemcpy(h_gamma, gamma, (M - 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
       hipMemcpy(h_other, other, (M - 1) * 4, hipMemcpyDeviceToHost) != hipSuccess))
    st = FDB_ERR_HIP;
  int32_t cnt = 0;
  if (st == FDB_OK && hipMemcpy(&cnt, count, 4, hipMemcpyDeviceToHost) != hipSuccess) st = FDB_ERR_HIP;
  if (st == FDB_OK && cnt > 0 &&
      hipMemcpy(h_leaves, leaves, static_cast<size_t>(cnt < m ? cnt : m) * 4, hipMemcpyDeviceToHost) != hipSuccess)
    st = FDB_ERR_HIP;
  uint32_t info = 0;
  if (st == FDB_OK && hipMemcpy(&info, h->d_info, 4, hipMemcpyDeviceToHost) != hipSuccess) st = FDB_ERR_HIP;
  if (st == FDB_OK && (info & FDB_INFO_INTERNAL)) st = FDB_ERR_INTERNAL;
  *h_num_leaves = cnt;
  (void)hipFree(buf);
  return st;
}

fdb_status fdb_set_timing(fdb_handle* h, int32_t enable) {
  if (!h) return FDB_ERR_INVALID;
  DeviceGuard g(h->device);
  fdb_status st = collect_timing(h);
  h->names.clear();
  h->ms.clear();
  h->timed_calls = 0;
  h->timing = enable != 0;
  return st;
}

fdb_status fdb_stage_times(fdb_handle* h, int32_t max, const char** h_names, double* h_ms, int32_t* h_count,
                           int32_t* h_calls) {
  if (!h || max < 0 || !h_count) return FDB_ERR_INVALID;
  DeviceGuard g(h->device);
  fdb_status st = collect_timing(h);
  if (st != FDB_OK) return st;
  int32_t k = static_cast<int32_t>(h->names.size());
  *h_count = k;
  for (int32_t i = 0; i < k && i < max; ++i) {
    if (h_names) h_names[i] = h->names[i].c_str();
    if (h_ms) h_ms[i] = h->ms[i];
  }
  if (h_calls) *h_calls = h->timed_calls;
  return FDB_OK;
}

fdb_status fdb_dbscan(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                      const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                      void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!h) return FDB_ERR_INVALID;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  return dbscan_entry(h, points, n, dim, eps, min_pts, opt, labels, is_core, h_num_clusters, workspace,
                      workspace_bytes, stream);
}

fdb_status fdb_dbscan_noalloc(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                              const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                              hipStream_t stream) {
  if (!h) return FDB_ERR_INVALID;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o) || (o.flags & FDB_FLAG_GRAPH)) return FDB_ERR_INVALID;  // instantiating a graph allocates
  if ((dim != 2 && dim != 3) || n < 0 || n > fdb::kMaxPoints) return FDB_ERR_INVALID;
  if (fdb::make_plan(n, dim, o.algo).bytes > FDB_NOALLOC_SCRATCH_BYTES) return FDB_ERR_SCRATCH;
  if (!h->scratch) return FDB_ERR_HIP;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  return dbscan_entry(h, points, n, dim, eps, min_pts, &o, labels, is_core, h_num_clusters, h->scratch,
                      FDB_NOALLOC_SCRATCH_BYTES, stream, false);
}

}  // extern "C"

namespace {

fdb_status dbscan_entry(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                        const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* h_num_clusters,
                        void* workspace, size_t workspace_bytes, hipStream_t stream, bool may_time) {
  using namespace fdb;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o)) return FDB_ERR_INVALID;
  if (dim != 2 && dim != 3) return FDB_ERR_INVALID;
  if (n < 0 || n > kMaxPoints) return FDB_ERR_INVALID;
  if (!std::isfinite(eps) || !(eps > 0.0f) || min_pts < 1) return FDB_ERR_INVALID;
  if (n > 0 && (!points || !labels)) return FDB_ERR_INVALID;
  DeviceGuard guard(h->device);
  h->last_stream = stream;
  h->host_info = 0;
  if (n == 0) {
    if (h_num_clusters) *h_num_clusters = 0;
    return FDB_OK;
  }
  resolve_shape(h, o, n, dim, 0, min_pts);
  const Plan plan = make_plan(n, dim, o.algo);
  void* ws = nullptr;
  const fdb_status wst = take_workspace(h, plan, workspace, workspace_bytes, stream, &ws);
  if (wst != FDB_OK) return wst;
  const SingleArgs args{points, n, dim, eps, min_pts, labels, is_core};
  fdb_status st;
  if (o.flags & FDB_FLAG_GRAPH) {
    const CallKey key = single_key(args, o, ws, plan.bytes);
    st = run_graph(h, key, stream, [&](hipStream_t cs) { return dbscan_launch(h, args, o, plan, ws, cs, false); });
    h->last_misc = at<int>(ws, plan.misc);
    h->last_densebox = o.algo != FDB_ALGO_FDBSCAN;
    h->last_n = n;
  } else {
    st = dbscan_launch(h, args, o, plan, ws, stream, h->timing && may_time);
  }
  if (st != FDB_OK) return st;
  if (h_num_clusters) {
    if (hipMemcpyAsync(h->h_pinned, at<int>(ws, plan.misc) + kMiscNumClusters, 4, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->h_pinned + 8, h->d_info, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return FDB_ERR_HIP;
    *h_num_clusters = static_cast<int32_t>(h->h_pinned[0]);
    if (h->h_pinned[8] & FDB_INFO_NONFINITE) return FDB_ERR_NONFINITE;
    if (h->h_pinned[8] & FDB_INFO_INTERNAL) return FDB_ERR_INTERNAL;
  }
  return FDB_OK;
}

// The launch sequence of one clustering call: stream-ordered launches only (no
// allocation, no host wait), so a stream capture can record it.
fdb_status dbscan_launch(fdb_handle* h, const SingleArgs& args, const fdb_options& o, const fdb::Plan& plan, void* ws,
                         hipStream_t stream, bool timing) {
  using namespace fdb;
  const float* points = args.points;
  const int64_t n = args.n;
  const int dim = args.dim;
  const float eps = args.eps;
  const int min_pts = args.min_pts;
  int32_t* labels = args.labels;
  uint8_t* is_core = args.is_core;
  const int leaf = o.leaf_size > 0 ? o.leaf_size : kDefaultLeaf;
  const int block = o.block_size > 0 ? o.block_size : kDefaultBlock;
  const int tile = o.tile > 0 ? o.tile : kDefaultTile;
  const bool densebox = o.algo != FDB_ALGO_FDBSCAN;  // the automatic choice is DenseBox
  const bool first_border = o.border == FDB_BORDER_FIRST;
  (void)hipGetLastError();
  const float eps2 = eps * eps;
  hipStream_t s = stream;
  Stager st(h, s, timing);
  if (timing) ++h->timed_calls;

  uint32_t* bounds = at<uint32_t>(ws, plan.bounds);
  int* misc = at<int>(ws, plan.misc);
  void* keys[2] = {at<void>(ws, plan.keys0), at<void>(ws, plan.keys1)};
  uint32_t* vals[2] = {at<uint32_t>(ws, plan.vals0), at<uint32_t>(ws, plan.vals1)};
  float* xs = at<float>(ws, plan.xs);
  int* lab = at<int>(ws, plan.labels);
  uint8_t* core = at<uint8_t>(ws, plan.core);

  st.mark("bounds");
  h->last_misc = misc;
  h->last_densebox = false;
  h->last_n = n;
  {
    // the call's counters and flags in one launch: info bits and the forest check's
    // count, the bounds' identities, the misc counters, and for DenseBox the digit
    // histograms, tile counters and look-back words of the planned sort
    FillList init;
    init.add(h->d_info, 0u, 2);
    init.add(bounds, 0xffffffffu, 4);
    init.add(bounds + 4, 0u, 4);
    init.add(misc, 0u, kMiscCount);
    if (densebox) {
      init.add(at<uint32_t>(ws, plan.hist), 0u, 8 * 256);
      init.add(at<uint32_t>(ws, plan.tilectr), 0u, 8);
      init.add(at<uint32_t>(ws, plan.status), 0u, planned_status_words(n));
    }
    fill_multi(init, s);
  }
  launch_bounds(points, n, dim, bounds, h->d_info, s);

  // DenseBox sizes its grid on the device (k_grid_plan): nothing waits for the GPU
  GridPlan* gplan = at<GridPlan>(ws, plan.gplan);
  if (densebox) launch_grid_plan(bounds, dim, eps, n, plan.map_bytes, gplan, h->d_info, s);

  int cur = 0;
  const uint32_t* perm = nullptr;
  TravArgs ta{};
  ta.xs = xs;
  ta.n = n;
  ta.eps2 = eps2;
  ta.packet_ext_eps2 = 9.0f;  // packet when the queries' box is at most 3 eps wide
  ta.packet_leaf = tile;       // buckets of up to `tile` candidates, one per lane
  ta.min_pts = min_pts;
  ta.labels = lab;
  ta.core = core;
  ta.cid = at<int>(ws, plan.cid);
  ta.border = at<int>(ws, plan.border);
  ta.block = block;
  ta.info = h->d_info;
  ta.t.node_a = at<float4>(ws, plan.node_a);
  ta.t.node_b = at<float4>(ws, plan.node_b);
  ta.t.rope = at<int>(ws, plan.rope);
  ta.t.leaf_rope = at<int>(ws, plan.leaf_rope);
  ta.t.leaf_size = leaf;

  if (densebox) {
    st.mark("cell_keys");
    launch_gridkeys(points, n, dim, bounds, gplan, keys[0], keys[1], vals[0], vals[1], at<uint32_t>(ws, plan.hist), s,
                    false);
    st.mark("sort");
    radix_sort_planned(keys[0], keys[1], vals[0], vals[1], n, gplan, at<uint32_t>(ws, plan.hist),
                       at<uint32_t>(ws, plan.digoff), at<uint32_t>(ws, plan.tilectr), at<uint64_t>(ws, plan.status),
                       h->d_info, s, false);
    cur = 1;  // the planned sort ends in buffer 1
    perm = vals[cur];
    st.mark("permute");
    launch_permute(points, n, dim, perm, xs, h->d_info, s);
    st.mark("dense_cells");
    densebox_cells(keys[cur], false, &gplan->key64, n, dim, xs, eps2, min_pts, at<int>(ws, plan.cell_id),
                   at<int>(ws, plan.cell_start), at<int>(ws, plan.cand), at<uint8_t>(ws, plan.cell_dense),
                   at<float4>(ws, plan.cell_lo), at<float4>(ws, plan.cell_hi), at<int>(ws, plan.pflag),
                   at<int>(ws, plan.prim_start), at<int>(ws, plan.prim_cnt),
                   at<float4>(ws, plan.prim_lo), at<float4>(ws, plan.prim_hi), at<uint64_t>(ws, plan.prim_key),
                   at<int>(ws, plan.dense_list), lab, core, misc, at<int>(ws, plan.bsums), plan.scan_blocks, s, 0,
                   nullptr, nullptr, at<int>(ws, plan.ends), at<int>(ws, plan.minorig));
  }
  h->last_densebox = densebox;
  if (densebox) {
    st.mark("lbvh");
    build_lbvh(at<void>(ws, plan.prim_key), true, static_cast<int>(n), dim, xs, n, at<float4>(ws, plan.prim_lo),
               at<float4>(ws, plan.prim_hi), at<float4>(ws, plan.node_a), at<float4>(ws, plan.node_b),
               at<int>(ws, plan.rope), at<int>(ws, plan.leaf_rope), at<int>(ws, plan.ends),
               at<int>(ws, plan.other), at<int>(ws, plan.gamma), misc + kMiscNumPrims, h->d_info, s,
               at<float4>(ws, plan.cut), misc + kMiscCut, true);
    ta.t.m_cap = static_cast<int>(n);
    ta.t.d_m = misc + kMiscNumPrims;
    ta.t.cut = at<float4>(ws, plan.cut);
    ta.t.cut_n = misc + kMiscCut;
    ta.prim_start = at<int>(ws, plan.prim_start);
    ta.prim_cnt = at<int>(ws, plan.prim_cnt);
    ta.prim_lo = at<float4>(ws, plan.prim_lo);
    ta.prim_hi = at<float4>(ws, plan.prim_hi);
    ta.dense_list = at<int>(ws, plan.dense_list);
    ta.d_ndense = misc + kMiscNumDense;
  } else {
    st.mark("morton");
    const int mbits = dim == 3 ? 63 : 62;
    launch_morton(points, n, dim, bounds, static_cast<uint64_t*>(keys[0]), vals[0], mbits,
                  at<uint32_t>(ws, plan.hist), s);
    st.mark("sort");
    cur = radix_sort(keys[0], keys[1], vals[0], vals[1], n, true, mbits, at<uint32_t>(ws, plan.hist), true,
                     at<uint32_t>(ws, plan.digoff), at<uint32_t>(ws, plan.tilectr), at<uint64_t>(ws, plan.status), h->d_info, s);
    perm = vals[cur];
    st.mark("permute");
    launch_permute(points, n, dim, perm, xs, h->d_info, s);
    launch_init_labels(lab, n, s, at<int>(ws, plan.ends), at<int>(ws, plan.minorig));
    st.mark("lbvh");
    build_lbvh(keys[cur], true, static_cast<int>(n), dim, xs, n, nullptr, nullptr, at<float4>(ws, plan.node_a),
               at<float4>(ws, plan.node_b), at<int>(ws, plan.rope), at<int>(ws, plan.leaf_rope),
               at<int>(ws, plan.ends), at<int>(ws, plan.other), at<int>(ws, plan.gamma),
               nullptr, h->d_info, s, at<float4>(ws, plan.cut), misc + kMiscCut, true, kCutDivFine);
    ta.t.m_cap = static_cast<int>(n);
    ta.t.d_m = nullptr;
    ta.t.cut = at<float4>(ws, plan.cut);
    ta.t.cut_n = misc + kMiscCut;
  }

  const bool all_core = min_pts <= 2;
  ta.lone = all_core ? nullptr : at<uint8_t>(ws, plan.lone);
  ta.qborder = at<int>(ws, plan.qborder);
  ta.qborder_n = misc + kMiscBorderQ;
  ta.brec_i = at<int>(ws, plan.brec_i);
  ta.brec_nb = at<int>(ws, plan.brec_nb);
  ta.brec_n = misc + kMiscBorderRec;
  ta.brec_cap = static_cast<int>(plan.brec_cap);
  if (!all_core) {
    // (the border counters are misc slots, cleared at the start of the call)
    // isolated points first, when the plan says the occupancy map fits the (now
    // free) cell-box buffers and its brick table the pflag buffer; otherwise these
    // kernels leave at once and the core pass walks every primitive
    if (densebox) {
      st.mark("isolated");
      ta.core_list = at<int>(ws, plan.cid);  // cid is free until the canonical ids
      ta.core_qn = misc + kMiscCoreQ;
      ta.lone_on = &gplan->lone_on;
      launch_lone_filter(ta, dim, at<uint64_t>(ws, plan.prim_key), gplan, at<uint32_t>(ws, plan.pflag),
                         at<uint64_t>(ws, plan.cell_lo), bounds, at<int>(ws, plan.cid), misc + kMiscCoreQ, s);
    }
    st.mark("core");
    launch_core(ta, dim, densebox, s);
  }
  if (densebox) {
    st.mark("main_cells");
    launch_main(ta, dim, true, all_core, first_border && !all_core, 1, s);
    st.mark("main_points");
    launch_main(ta, dim, true, all_core, first_border && !all_core, 2, s);
  } else {
    st.mark("main");
    if (all_core || !first_border) {
      // the packet main phase: core pairs of curve neighbours first, then per cut
      // subtree the set its core points are in, so packets pass over subtrees
      // already in their own set
      int* csum = reinterpret_cast<int*>(at<float4>(ws, plan.cut) + 2 * kCutMax);
      launch_fdb_local(ta, dim, all_core, s);
      launch_cut_summary(ta, all_core, csum, s);
      ta.t.cut_sum = csum;
      launch_main(ta, dim, false, all_core, false, 0, s);
    } else {
      launch_main(ta, dim, false, all_core, first_border && !all_core, 0, s);
    }
    ta.t.cut_sum = nullptr;
  }
  if (o.flags & FDB_FLAG_VALIDATE) launch_check_forest(lab, all_core ? nullptr : core, n, h->d_info + 1, h->d_info, s);
  st.mark("finalize");
  // with final core flags the pass also takes each cluster's smallest input index
  if (all_core) launch_finalize(lab, n, h->d_info, s);
  else launch_finalize(lab, n, h->d_info, s, core, perm, at<int>(ws, plan.minorig), at<uint32_t>(ws, plan.lflag), false);
  if (all_core) launch_core_from_sets(lab, core, n, min_pts, s);
  st.mark("cluster_ids");
  canonical_ids(lab, core, perm, n, at<int>(ws, plan.minorig), at<uint32_t>(ws, plan.lflag), at<int>(ws, plan.rank),
                at<int>(ws, plan.bsums), plan.scan_blocks, at<int>(ws, plan.cid), misc + kMiscNumClusters, s, true,
                !all_core);
  const bool have_border = !all_core && o.border == FDB_BORDER_CANONICAL;  // DBSCAN*: non-core stays noise
  if (have_border) {
    st.mark("border");
    launch_border(ta, dim, densebox, s);
  }
  st.mark("scatter");
  launch_scatter(lab, core, perm, at<int>(ws, plan.cid), at<int>(ws, plan.border), first_border && !all_core,
                 have_border, n, labels, is_core, h->d_info, s);
  st.finish();
  return hipGetLastError() == hipSuccess ? FDB_OK : FDB_ERR_HIP;
}

}  // namespace

namespace fdb {

const uint32_t* handle_info(const fdb_handle* h) { return h->d_info; }

}  // namespace fdb

extern "C" {

fdb_status fdb_workspace_bytes_batched(int64_t n_total, int32_t num_clouds, int32_t dim, const fdb_options* opt,
                                       size_t* h_out) {
  if (!h_out) return FDB_ERR_INVALID;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o) || (dim != 2 && dim != 3) || n_total < 0 || n_total > fdb::kMaxPoints || num_clouds < 1 ||
      num_clouds > (1 << 24))
    return FDB_ERR_INVALID;
  *h_out = fdb::make_plan(n_total, dim, o.algo, num_clouds).bytes;
  return FDB_OK;
}

fdb_status fdb_dbscan_batched(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                              int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                              const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* num_clusters,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!h) return FDB_ERR_INVALID;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  return dbscan_batched_entry(h, points, n_total, offsets, num_clouds, dim, eps, min_pts, opt, labels, is_core,
                              num_clusters, workspace, workspace_bytes, stream);
}

}  // extern "C"

namespace {

fdb_status dbscan_batched_entry(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                                int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                                const fdb_options* opt, int32_t* labels, uint8_t* is_core, int32_t* num_clusters,
                                void* workspace, size_t workspace_bytes, hipStream_t stream) {
  using namespace fdb;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o) || (dim != 2 && dim != 3) || n_total < 0 || n_total > kMaxPoints || num_clouds < 1 ||
      num_clouds > (1 << 24) || !offsets || !eps || !min_pts)
    return FDB_ERR_INVALID;
  if (n_total > 0 && (!points || !labels)) return FDB_ERR_INVALID;
  DeviceGuard guard(h->device);
  h->last_stream = stream;
  h->host_info = 0;
  h->last_misc = nullptr;
  if (n_total == 0) {
    if (num_clusters) fill_u32(reinterpret_cast<uint32_t*>(num_clusters), 0, num_clouds, stream);
    return hipGetLastError() == hipSuccess ? FDB_OK : FDB_ERR_HIP;
  }
  resolve_shape(h, o, n_total, dim, num_clouds);
  const Plan plan = make_plan(n_total, dim, o.algo, num_clouds);
  void* ws = nullptr;
  const fdb_status wst = take_workspace(h, plan, workspace, workspace_bytes, stream, &ws);
  if (wst != FDB_OK) return wst;
  const BatchArgs args{points, n_total, offsets, num_clouds, dim, eps, min_pts, labels, is_core, num_clusters};
  if (o.flags & FDB_FLAG_GRAPH) {
    const CallKey key = batch_key(args, o, ws, plan.bytes);
    const fdb_status st =
        run_graph(h, key, stream, [&](hipStream_t cs) { return batched_launch(h, args, o, plan, ws, cs, false); });
    h->last_misc = at<int>(ws, plan.misc);
    h->last_densebox = o.algo != FDB_ALGO_FDBSCAN;
    h->last_n = n_total;
    return st;
  }
  return batched_launch(h, args, o, plan, ws, stream, h->timing);
}

// The launch sequence of one batched call (stream-ordered launches only).
fdb_status batched_launch(fdb_handle* h, const BatchArgs& args, const fdb_options& o, const fdb::Plan& plan, void* ws,
                          hipStream_t stream, bool timing) {
  using namespace fdb;
  const float* points = args.points;
  const int64_t n_total = args.n_total;
  const int64_t* offsets = args.offsets;
  const int32_t num_clouds = args.num_clouds;
  const int dim = args.dim;
  const float* eps = args.eps;
  const int32_t* min_pts = args.min_pts;
  int32_t* labels = args.labels;
  uint8_t* is_core = args.is_core;
  int32_t* num_clusters = args.num_clusters;
  hipStream_t s = stream;
  const int leaf = o.leaf_size > 0 ? o.leaf_size : kDefaultLeaf;
  const int block = o.block_size > 0 ? o.block_size : kDefaultBlock;
  const int tile = o.tile > 0 ? o.tile : kDefaultTile;
  const bool densebox = o.algo != FDB_ALGO_FDBSCAN;  // the automatic choice runs DenseBox for a batch
  const bool first_border = o.border == FDB_BORDER_FIRST;
  (void)hipGetLastError();
  Stager st(h, s, timing);
  if (timing) ++h->timed_calls;
  const int64_t n = n_total;
  int cb = 1;
  while ((int64_t(1) << cb) < num_clouds) ++cb;
  const int bpd = std::min(dim == 3 ? 21 : 31, (64 - cb) / dim);  // key bits per axis below the cloud id
  const int shift = dim * bpd;
  int* misc = at<int>(ws, plan.misc);
  h->last_misc = misc;  // fdb_last_counts reports the batch as a whole
  h->last_densebox = densebox;
  h->last_n = n;
  void* keys[2] = {at<void>(ws, plan.keys0), at<void>(ws, plan.keys1)};
  uint32_t* vals[2] = {at<uint32_t>(ws, plan.vals0), at<uint32_t>(ws, plan.vals1)};
  float* xs = at<float>(ws, plan.xs);
  int* lab = at<int>(ws, plan.labels);
  uint8_t* core = at<uint8_t>(ws, plan.core);
  float4* cl_lo = at<float4>(ws, plan.cl_lo);
  float4* cl_scale = at<float4>(ws, plan.cl_scale);
  float* cl_eps2 = at<float>(ws, plan.cl_eps2);
  int* cl_minpts = at<int>(ws, plan.cl_minpts);
  int* cl_root = at<int>(ws, plan.cl_root);
  int* cl_end = at<int>(ws, plan.cl_end);

  st.mark("clouds");
  fill_u32(h->d_info, 0, 2, s);  // info bits and the forest check's count
  fill_u32(reinterpret_cast<uint32_t*>(misc), 0, kMiscCount, s);
  int* cl_flags = at<int>(ws, plan.cl_flags);
  batch_prep(points, offsets, num_clouds, n, dim, eps, min_pts, bpd, densebox, at<uint32_t>(ws, plan.cl_ord), cl_lo,
             cl_scale, cl_eps2, cl_minpts, cl_flags, h->d_info, s);
  st.mark("keys");
  batch_keys(points, offsets, num_clouds, n, dim, cl_lo, cl_scale, bpd, shift, static_cast<uint64_t*>(keys[0]),
             vals[0], shift + cb, at<uint32_t>(ws, plan.hist), s);
  st.mark("sort");
  const int cur = radix_sort(keys[0], keys[1], vals[0], vals[1], n, true, shift + cb, at<uint32_t>(ws, plan.hist), true,
                             at<uint32_t>(ws, plan.digoff), at<uint32_t>(ws, plan.tilectr),
                             at<uint64_t>(ws, plan.status), h->d_info, s);
  const uint32_t* perm = vals[cur];
  const uint64_t* pkeys = static_cast<const uint64_t*>(keys[cur]);
  st.mark("permute");
  launch_permute(points, n, dim, perm, xs, h->d_info, s);

  TravArgs ta{};
  ta.xs = xs;
  ta.n = n;
  ta.eps2 = 0.0f;
  ta.packet_ext_eps2 = 9.0f;
  ta.packet_leaf = tile;
  ta.min_pts = 0;
  ta.labels = lab;
  ta.core = core;
  ta.cid = at<int>(ws, plan.cid);
  ta.border = at<int>(ws, plan.border);
  ta.block = block;
  ta.info = h->d_info;
  ta.t.node_a = at<float4>(ws, plan.node_a);
  ta.t.node_b = at<float4>(ws, plan.node_b);
  ta.t.rope = at<int>(ws, plan.rope);
  ta.t.leaf_rope = at<int>(ws, plan.leaf_rope);
  ta.t.leaf_size = leaf;
  ta.t.m_cap = static_cast<int>(n);
  ta.pkeys = pkeys;
  ta.key_shift = shift;
  ta.num_clouds = num_clouds;
  ta.cloud_root = cl_root;
  ta.cloud_end = cl_end;
  ta.cloud_eps2 = cl_eps2;
  ta.cloud_minpts = cl_minpts;

  if (densebox) {
    st.mark("dense_cells");
    densebox_cells(keys[cur], true, nullptr, n, dim, xs, 0.0f, 0, at<int>(ws, plan.cell_id), at<int>(ws, plan.cell_start),
                   at<int>(ws, plan.cand), at<uint8_t>(ws, plan.cell_dense), at<float4>(ws, plan.cell_lo),
                   at<float4>(ws, plan.cell_hi), at<int>(ws, plan.pflag),
                   at<int>(ws, plan.prim_start), at<int>(ws, plan.prim_cnt), at<float4>(ws, plan.prim_lo),
                   at<float4>(ws, plan.prim_hi), at<uint64_t>(ws, plan.prim_key), at<int>(ws, plan.dense_list), lab,
                   core, misc, at<int>(ws, plan.bsums), plan.scan_blocks, s, shift, cl_minpts, cl_eps2,
                   at<int>(ws, plan.ends), at<int>(ws, plan.minorig));
    st.mark("lbvh");
    build_lbvh(at<void>(ws, plan.prim_key), true, static_cast<int>(n), dim, xs, n, at<float4>(ws, plan.prim_lo),
               at<float4>(ws, plan.prim_hi), at<float4>(ws, plan.node_a), at<float4>(ws, plan.node_b),
               at<int>(ws, plan.rope), at<int>(ws, plan.leaf_rope), at<int>(ws, plan.ends),
               at<int>(ws, plan.other), at<int>(ws, plan.gamma), misc + kMiscNumPrims, h->d_info, s, nullptr,
               nullptr, true);
    batch_roots(offsets, num_clouds, n, at<int>(ws, plan.cand), misc + kMiscNumPrims, at<int>(ws, plan.other),
                cl_root, cl_end, h->d_info, s);
    ta.t.d_m = misc + kMiscNumPrims;
    ta.prim_start = at<int>(ws, plan.prim_start);
    ta.prim_cnt = at<int>(ws, plan.prim_cnt);
    ta.prim_lo = at<float4>(ws, plan.prim_lo);
    ta.prim_hi = at<float4>(ws, plan.prim_hi);
    ta.dense_list = at<int>(ws, plan.dense_list);
    ta.d_ndense = misc + kMiscNumDense;
  } else {
    launch_init_labels(lab, n, s, at<int>(ws, plan.ends), at<int>(ws, plan.minorig));
    st.mark("lbvh");
    build_lbvh(keys[cur], true, static_cast<int>(n), dim, xs, n, nullptr, nullptr, at<float4>(ws, plan.node_a),
               at<float4>(ws, plan.node_b), at<int>(ws, plan.rope), at<int>(ws, plan.leaf_rope),
               at<int>(ws, plan.ends), at<int>(ws, plan.other), at<int>(ws, plan.gamma),
               nullptr, h->d_info, s, nullptr, nullptr, true);
    batch_roots(offsets, num_clouds, n, nullptr, nullptr, at<int>(ws, plan.other), cl_root, cl_end, h->d_info, s);
    ta.t.d_m = nullptr;
  }
  st.mark("core");
  ta.lone = at<uint8_t>(ws, plan.lone);
  ta.qborder = at<int>(ws, plan.qborder);
  ta.qborder_n = misc + kMiscBorderQ;
  ta.brec_i = at<int>(ws, plan.brec_i);
  ta.brec_nb = at<int>(ws, plan.brec_nb);
  ta.brec_n = misc + kMiscBorderRec;
  ta.brec_cap = static_cast<int>(plan.brec_cap);
  launch_core(ta, dim, densebox, s);
  if (densebox) {
    st.mark("main_cells");
    launch_main(ta, dim, true, false, first_border, 1, s);
    st.mark("main_points");
    launch_main(ta, dim, true, false, first_border, 2, s);
  } else {
    st.mark("main");
    launch_main(ta, dim, false, false, first_border, 0, s);
  }
  if (o.flags & FDB_FLAG_VALIDATE) launch_check_forest(lab, core, n, h->d_info + 1, h->d_info, s);
  st.mark("finalize");
  // batches run the core pass
  launch_finalize(lab, n, h->d_info, s, core, perm, at<int>(ws, plan.minorig), at<uint32_t>(ws, plan.lflag), false);
  st.mark("cluster_ids");
  int* rank = at<int>(ws, plan.rank);
  uint32_t* lbits = at<uint32_t>(ws, plan.lflag);
  canonical_ids(lab, core, perm, n, at<int>(ws, plan.minorig), lbits, rank, at<int>(ws, plan.bsums),
                plan.scan_blocks, at<int>(ws, plan.cid), misc + kMiscNumClusters, s, false, true);
  batch_cluster_ids(lab, core, at<int>(ws, plan.minorig), lbits, rank, pkeys, shift, offsets, num_clouds, n,
                    misc + kMiscNumClusters, cl_flags, at<int>(ws, plan.cid), num_clusters, s);
  if (o.border == FDB_BORDER_CANONICAL) {
    st.mark("border");
    launch_border(ta, dim, densebox, s);
  }
  st.mark("scatter");
  launch_scatter(lab, core, perm, at<int>(ws, plan.cid), at<int>(ws, plan.border), first_border,
                 o.border == FDB_BORDER_CANONICAL, n,
                 labels, is_core, h->d_info, s);
  st.finish();
  return hipGetLastError() == hipSuccess ? FDB_OK : FDB_ERR_HIP;
}

}  // namespace

extern "C" {


// ---- out-of-core batches --------------------------------------------------------

namespace {

// Device bytes of one group slot: its batched workspace, points, offsets, eps,
// minPts, K, labels and core flags.
size_t ooc_slot_bytes(int64_t n, int32_t b, int dim, int algo) {
  const fdb::Plan plan = fdb::make_plan(n, dim, algo, b);
  return fdb::align_up(plan.bytes) + fdb::align_up(size_t(n) * dim * 4) + fdb::align_up(size_t(b + 1) * 8) +
         3 * fdb::align_up(size_t(b) * 4) + fdb::align_up(size_t(n) * 4) + fdb::align_up(size_t(n));
}

struct OocSlot {
  void* base = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  float* pts = nullptr;
  int64_t* off = nullptr;
  float* eps = nullptr;
  int32_t* mp = nullptr;
  int32_t* k = nullptr;
  int32_t* lab = nullptr;
  uint8_t* core = nullptr;
  int64_t* h_off = nullptr;   // pinned: the group's offsets, rebased to its first point
  uint32_t* h_info = nullptr; // pinned: the group's FDB_INFO_* bits
  hipEvent_t h2d = nullptr, comp = nullptr, d2h = nullptr;
};

}  // namespace

fdb_status fdb_dbscan_batched_host(fdb_handle* h, const float* h_points, const int64_t* h_offsets,
                                   int32_t num_clouds, int32_t dim, const float* h_eps, const int32_t* h_min_pts,
                                   const fdb_options* opt, size_t device_budget_bytes, int32_t* h_labels,
                                   uint8_t* h_is_core, int32_t* h_num_clusters) {
  using namespace fdb;
  if (!h || !h_offsets || !h_eps || !h_min_pts || !h_num_clusters || (dim != 2 && dim != 3) || num_clouds < 1 ||
      num_clouds > (1 << 24))
    return FDB_ERR_INVALID;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o) || h_offsets[0] != 0) return FDB_ERR_INVALID;
  for (int32_t c = 0; c < num_clouds; ++c)
    if (h_offsets[c + 1] < h_offsets[c]) return FDB_ERR_INVALID;
  const int64_t n_total = h_offsets[num_clouds];
  if (n_total > 0 && (!h_points || !h_labels)) return FDB_ERR_INVALID;

  // Groups of consecutive whole clouds, each filling at most half the budget
  // (two slots: one group is copied in while the other is clustered).
  const size_t cap = (device_budget_bytes / 2) & ~size_t(255);
  std::vector<int32_t> gbeg;
  int64_t gn = 0;
  int32_t b_max = 0;
  size_t slot_bytes = 0;  // the largest group's footprint; each group is carved from its slot on its own
  gbeg.push_back(0);
  for (int32_t c = 0; c < num_clouds; ++c) {
    const int64_t nc = h_offsets[c + 1] - h_offsets[c];
    if (nc > kMaxPoints) return FDB_ERR_INVALID;
    if (ooc_slot_bytes(nc, 1, dim, o.algo) > cap) return FDB_ERR_NOMEM;  // a cloud alone does not fit
    const int32_t b = c - gbeg.back();
    if (b > 0 && (gn + nc > kMaxPoints || ooc_slot_bytes(gn + nc, b + 1, dim, o.algo) > cap)) {
      slot_bytes = std::max(slot_bytes, ooc_slot_bytes(gn, b, dim, o.algo));
      b_max = std::max(b_max, b);
      gbeg.push_back(c);
      gn = 0;
    }
    gn += nc;
  }
  slot_bytes = std::max(slot_bytes, ooc_slot_bytes(gn, num_clouds - gbeg.back(), dim, o.algo));
  b_max = std::max(b_max, num_clouds - gbeg.back());
  gbeg.push_back(num_clouds);
  const size_t groups = gbeg.size() - 1;

  DeviceGuard guard(h->device);
  OocSlot slot[2];
  hipStream_t sc = nullptr, sk = nullptr;  // clustering, copies
  fdb_status st = FDB_OK;
  uint32_t info = 0;
  auto fail = [&](fdb_status e) {
    if (st == FDB_OK) st = e;
  };
  if (hipStreamCreateWithFlags(&sc, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sk, hipStreamNonBlocking) != hipSuccess)
    fail(FDB_ERR_HIP);
  for (int k = 0; k < 2 && st == FDB_OK; ++k) {
    OocSlot& S = slot[k];
    if (hipMalloc(&S.base, slot_bytes) != hipSuccess) {
      S.base = nullptr;
      fail(FDB_ERR_NOMEM);
      break;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&S.h_off), size_t(b_max + 1) * 8 + 256, hipHostMallocDefault) !=
        hipSuccess) {
      S.h_off = nullptr;
      fail(FDB_ERR_NOMEM);
      break;
    }
    S.h_info = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(S.h_off) + align_up(size_t(b_max + 1) * 8));
    *S.h_info = 0;
    if (hipEventCreateWithFlags(&S.h2d, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S.comp, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S.d2h, hipEventDisableTiming) != hipSuccess)
      fail(FDB_ERR_HIP);
  }

  // Results of group g back to the caller (copy stream, after its clustering).
  auto copy_out = [&](size_t g) {
    OocSlot& S = slot[g & 1];
    const int32_t c0 = gbeg[g], b = gbeg[g + 1] - c0;
    const int64_t p0 = h_offsets[c0], n = h_offsets[gbeg[g + 1]] - p0;
    if (hipStreamWaitEvent(sk, S.comp, 0) != hipSuccess) return fail(FDB_ERR_HIP);
    if ((n > 0 && hipMemcpyAsync(h_labels + p0, S.lab, size_t(n) * 4, hipMemcpyDeviceToHost, sk) != hipSuccess) ||
        (n > 0 && h_is_core &&
         hipMemcpyAsync(h_is_core + p0, S.core, size_t(n), hipMemcpyDeviceToHost, sk) != hipSuccess) ||
        hipMemcpyAsync(h_num_clusters + c0, S.k, size_t(b) * 4, hipMemcpyDeviceToHost, sk) != hipSuccess ||
        hipEventRecord(S.d2h, sk) != hipSuccess)
      fail(FDB_ERR_HIP);
  };
  for (size_t g = 0; g < groups && st == FDB_OK; ++g) {
    OocSlot& S = slot[g & 1];
    if (g >= 2) {  // the slot's previous group has left it
      if (hipEventSynchronize(S.d2h) != hipSuccess) {
        fail(FDB_ERR_HIP);
        break;
      }
      info |= *S.h_info;
    }
    const int32_t c0 = gbeg[g], b = gbeg[g + 1] - c0;
    const int64_t p0 = h_offsets[c0], n = h_offsets[gbeg[g + 1]] - p0;
    {  // this group's layout in its slot (at most ooc_slot_bytes(n, b) <= slot_bytes)
      char* q = static_cast<char*>(S.base);
      auto take = [&](size_t bytes) {
        char* r = q;
        q += align_up(bytes);
        return r;
      };
      S.ws_bytes = align_up(make_plan(n, dim, o.algo, b).bytes);
      S.ws = take(S.ws_bytes);
      S.pts = reinterpret_cast<float*>(take(size_t(n) * dim * 4));
      S.off = reinterpret_cast<int64_t*>(take(size_t(b + 1) * 8));
      S.eps = reinterpret_cast<float*>(take(size_t(b) * 4));
      S.mp = reinterpret_cast<int32_t*>(take(size_t(b) * 4));
      S.k = reinterpret_cast<int32_t*>(take(size_t(b) * 4));
      S.lab = reinterpret_cast<int32_t*>(take(size_t(n) * 4));
      S.core = reinterpret_cast<uint8_t*>(take(size_t(n)));
    }
    for (int32_t c = 0; c <= b; ++c) S.h_off[c] = h_offsets[c0 + c] - p0;
    if ((n > 0 && hipMemcpyAsync(S.pts, h_points + p0 * dim, size_t(n) * dim * 4, hipMemcpyHostToDevice, sk) !=
                      hipSuccess) ||
        hipMemcpyAsync(S.off, S.h_off, size_t(b + 1) * 8, hipMemcpyHostToDevice, sk) != hipSuccess ||
        hipMemcpyAsync(S.eps, h_eps + c0, size_t(b) * 4, hipMemcpyHostToDevice, sk) != hipSuccess ||
        hipMemcpyAsync(S.mp, h_min_pts + c0, size_t(b) * 4, hipMemcpyHostToDevice, sk) != hipSuccess ||
        hipEventRecord(S.h2d, sk) != hipSuccess || hipStreamWaitEvent(sc, S.h2d, 0) != hipSuccess) {
      fail(FDB_ERR_HIP);
      break;
    }
    const fdb_status r = dbscan_batched_entry(h, S.pts, n, S.off, b, dim, S.eps, S.mp, &o, S.lab,
                                              h_is_core ? S.core : nullptr, S.k, S.ws, S.ws_bytes, sc);
    if (r != FDB_OK) {
      fail(r);
      break;
    }
    if (hipMemcpyAsync(S.h_info, h->d_info, 4, hipMemcpyDeviceToHost, sc) != hipSuccess ||
        hipEventRecord(S.comp, sc) != hipSuccess) {
      fail(FDB_ERR_HIP);
      break;
    }
    // queued behind this group's input copies, so they overlap the previous group's clustering
    if (g >= 1) copy_out(g - 1);
  }
  if (st == FDB_OK && groups > 0) copy_out(groups - 1);
  if (sc && hipStreamSynchronize(sc) != hipSuccess) fail(FDB_ERR_HIP);
  if (sk && hipStreamSynchronize(sk) != hipSuccess) fail(FDB_ERR_HIP);
  if (st == FDB_OK)
    for (size_t g = groups >= 2 ? groups - 2 : 0; g < groups; ++g) info |= *slot[g & 1].h_info;
  for (OocSlot& S : slot) {
    if (S.h2d) (void)hipEventDestroy(S.h2d);
    if (S.comp) (void)hipEventDestroy(S.comp);
    if (S.d2h) (void)hipEventDestroy(S.d2h);
    if (S.h_off) (void)hipHostFree(S.h_off);
    if (S.base) (void)hipFree(S.base);
  }
  if (sc) (void)hipStreamDestroy(sc);
  if (sk) (void)hipStreamDestroy(sk);
  // fdb_last_info / fdb_last_counts now describe this call as a whole
  h->last_stream = nullptr;
  h->last_misc = nullptr;
  h->host_info = info;
  if (st == FDB_OK && (info & FDB_INFO_INTERNAL)) st = FDB_ERR_INTERNAL;
  return st;
}

// ---- autotuner ------------------------------------------------------------------
//
// The launch shape (leaf size, workgroup size, traversal tile) changes no label,
// only time. fdb_tune times candidate shapes on the caller's own input by
// coordinate descent (each axis over its candidates, the others held at the best
// so far), keeps the fastest for the call's class and appends it to the file
// named by FDB_TUNE_CACHE, which fdb_create reads back.

}  // extern "C"

namespace {

constexpr int kTuneLeaf[] = {4, 8, 16, 32};
constexpr int kTuneBlock[] = {64, 128, 256};
constexpr int kTuneTile[] = {32, 64};

void store_tune(fdb_handle* h, const fdb::TuneEntry& e) {
  for (auto& x : h->tune)
    if (x.batched == e.batched && x.algo == e.algo && x.dim == e.dim && x.nlog2 == e.nlog2 &&
        x.mpclass == e.mpclass) {
      x = e;
      return;
    }
  h->tune.push_back(e);
}

void append_tune_file(const fdb::TuneEntry& e) {
  const char* path = std::getenv("FDB_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "fdbtune1 %d %d %d %d %d %d %d %d %.6f %.6f %.6f\n", e.batched, e.algo, e.dim, e.nlog2, e.mpclass,
               e.leaf_size, e.block_size, e.tile, e.best_ms, e.default_ms, e.dense_share);
  std::fclose(f);
}

// Later lines override earlier ones for the same class; malformed lines are skipped.
void load_tune_file(fdb_handle* h) {
  const char* path = std::getenv("FDB_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    fdb::TuneEntry e{};
    if (std::sscanf(line, "fdbtune1 %d %d %d %d %d %d %d %d %lf %lf %lf", &e.batched, &e.algo, &e.dim, &e.nlog2,
                    &e.mpclass, &e.leaf_size, &e.block_size, &e.tile, &e.best_ms, &e.default_ms,
                    &e.dense_share) != 11)
      continue;
    fdb_options o{};
    o.leaf_size = e.leaf_size;
    o.block_size = e.block_size;
    o.tile = e.tile;
    if (!valid_options(o) || e.leaf_size < 1 || (e.dim != 2 && e.dim != 3)) continue;
    store_tune(h, e);
  }
  std::fclose(f);
}

// Median time (ms) of `reps` runs of call(o) on `stream`, timed with HIP events.
template <typename F>
fdb_status time_shape(hipStream_t stream, int reps, const fdb_options& o, F&& call, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return FDB_ERR_HIP;
  }
  fdb_status st = call(o);  // warm-up (and the first graph recording, if asked for)
  std::vector<double> t;
  for (int r = 0; r < reps && st == FDB_OK; ++r) {
    float x = 0.0f;
    if (hipEventRecord(a, stream) != hipSuccess) st = FDB_ERR_HIP;
    if (st == FDB_OK) st = call(o);
    if (st == FDB_OK && (hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                         hipEventElapsedTime(&x, a, b) != hipSuccess))
      st = FDB_ERR_HIP;
    t.push_back(x);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != FDB_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return FDB_OK;
}

template <typename F>
fdb_status tune_search(fdb_handle* h, hipStream_t stream, int reps, const fdb_options& base, F&& call,
                       fdb_options* best, double* best_ms, double* default_ms) {
  fdb_options cur = base;
  cur.leaf_size = kDefaultLeaf;
  cur.block_size = kDefaultBlock;
  cur.tile = kDefaultTile;
  double cur_ms = 0.0;
  fdb_status st = time_shape(stream, reps, cur, call, &cur_ms);
  if (st != FDB_OK) return st;
  *default_ms = cur_ms;
  auto axis = [&](int32_t fdb_options::*field, const int* cand, int count) -> fdb_status {
    for (int k = 0; k < count; ++k) {
      if (cur.*field == cand[k]) continue;
      fdb_options o = cur;
      o.*field = cand[k];
      double ms = 0.0;
      const fdb_status r = time_shape(stream, reps, o, call, &ms);
      if (r != FDB_OK) return r;
      if (ms < cur_ms) {
        cur = o;
        cur_ms = ms;
      }
    }
    return FDB_OK;
  };
  if ((st = axis(&fdb_options::leaf_size, kTuneLeaf, 4)) != FDB_OK) return st;
  if ((st = axis(&fdb_options::block_size, kTuneBlock, 3)) != FDB_OK) return st;
  if ((st = axis(&fdb_options::tile, kTuneTile, 2)) != FDB_OK) return st;
  *best = cur;
  *best_ms = cur_ms;
  (void)h;
  return FDB_OK;
}

double dense_share_of(fdb_handle* h, int64_t n) {
  int64_t c[4];
  if (n <= 0 || fdb_last_counts(h, c) != FDB_OK || c[2] <= 0) return 0.0;
  return static_cast<double>(n - (c[3] - c[2])) / static_cast<double>(n);
}

}  // namespace

extern "C" {

fdb_status fdb_tune(fdb_handle* h, const float* points, int64_t n, int32_t dim, float eps, int32_t min_pts,
                    const fdb_options* opt, int32_t reps, int32_t* labels, uint8_t* is_core, void* workspace,
                    size_t workspace_bytes, hipStream_t stream, fdb_options* h_best, double* h_ms) {
  if (!h || !h_best || !h_ms || reps < 1 || reps > 100 || n < 1) return FDB_ERR_INVALID;
  fdb_options base{};
  if (opt) base = *opt;
  if (!valid_options(base)) return FDB_ERR_INVALID;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  DeviceGuard guard(h->device);
  auto call = [&](const fdb_options& o) {
    return dbscan_entry(h, points, n, dim, eps, min_pts, &o, labels, is_core, nullptr, workspace, workspace_bytes,
                        stream);
  };
  fdb_options best{};
  double best_ms = 0.0, def_ms = 0.0;
  const fdb_status st = tune_search(h, stream, reps, base, call, &best, &best_ms, &def_ms);
  if (st != FDB_OK) return st;
  fdb::TuneEntry e{0, base.algo == FDB_ALGO_FDBSCAN ? FDB_ALGO_FDBSCAN : FDB_ALGO_DENSEBOX, dim, nlog2_of(n),
                   mpclass_of(min_pts), best.leaf_size, best.block_size, best.tile, best_ms, def_ms,
                   dense_share_of(h, n)};
  store_tune(h, e);
  append_tune_file(e);
  *h_best = best;
  h_ms[0] = best_ms;
  h_ms[1] = def_ms;
  return FDB_OK;
}

fdb_status fdb_tune_batched(fdb_handle* h, const float* points, int64_t n_total, const int64_t* offsets,
                            int32_t num_clouds, int32_t dim, const float* eps, const int32_t* min_pts,
                            const fdb_options* opt, int32_t reps, int32_t* labels, uint8_t* is_core,
                            int32_t* num_clusters, void* workspace, size_t workspace_bytes, hipStream_t stream,
                            fdb_options* h_best, double* h_ms) {
  if (!h || !h_best || !h_ms || reps < 1 || reps > 100 || n_total < 1) return FDB_ERR_INVALID;
  fdb_options base{};
  if (opt) base = *opt;
  if (!valid_options(base)) return FDB_ERR_INVALID;
  CallGuard busy(h);
  if (!busy.ok) return FDB_ERR_BUSY;
  DeviceGuard guard(h->device);
  auto call = [&](const fdb_options& o) {
    return dbscan_batched_entry(h, points, n_total, offsets, num_clouds, dim, eps, min_pts, &o, labels, is_core,
                                num_clusters, workspace, workspace_bytes, stream);
  };
  fdb_options best{};
  double best_ms = 0.0, def_ms = 0.0;
  const fdb_status st = tune_search(h, stream, reps, base, call, &best, &best_ms, &def_ms);
  if (st != FDB_OK) return st;
  fdb::TuneEntry e{1, base.algo == FDB_ALGO_FDBSCAN ? FDB_ALGO_FDBSCAN : FDB_ALGO_DENSEBOX, dim, nlog2_of(n_total), 1,
                   best.leaf_size, best.block_size, best.tile, best_ms, def_ms, dense_share_of(h, n_total)};
  store_tune(h, e);
  append_tune_file(e);
  *h_best = best;
  h_ms[0] = best_ms;
  h_ms[1] = def_ms;
  return FDB_OK;
}

fdb_status fdb_tuned_options(fdb_handle* h, int64_t n, int32_t dim, int32_t min_pts, int32_t num_clouds,
                             const fdb_options* opt, fdb_options* h_out) {
  if (!h || !h_out || n < 0 || (dim != 2 && dim != 3) || num_clouds < 0) return FDB_ERR_INVALID;
  fdb_options o{};
  if (opt) o = *opt;
  if (!valid_options(o)) return FDB_ERR_INVALID;
  resolve_shape(h, o, n, dim, num_clouds, min_pts);
  if (!o.leaf_size) o.leaf_size = kDefaultLeaf;
  if (!o.block_size) o.block_size = kDefaultBlock;
  if (!o.tile) o.tile = kDefaultTile;
  *h_out = o;
  return FDB_OK;
}

}  // extern "C"
