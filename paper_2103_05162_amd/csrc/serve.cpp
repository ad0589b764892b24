// Served clustering. Jobs arrive one at a time, each with its own device
// buffers, eps and minPts. In batched mode the arena is split into kSlots slots,
// each with its own stream, handle, pinned mirror and completion event; a worker
// thread fills any free slot with the jobs waiting in the queue, oldest first, as
// long as the batch fits in the slot, and launches them as one batched launch
// sequence without waiting for it. So while one batch runs on the device, the
// jobs that arrived meanwhile are gathered and clustered in the other slot
// (continuous batching: admission as slots and memory free up, overlapping work).
// A slot is handed back when its event has fired. The budget is allocated once,
// when the server is created; nothing is allocated per job. In FIFO mode the
// worker runs one job at a time with fdb_dbscan in the whole arena, the plain
// server the batched one is compared with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "fdb_internal.hpp"
#include "fdbscan.h"

namespace {

using fdb::JobSeg;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Job {
  fdb_job in;
  int64_t t_submit = 0, t_start = 0, t_done = 0;
  int32_t state = 0;  // 0 queued, 1 running, 2 done
  int32_t status = FDB_OK;
  int32_t num_clusters = 0;
  int32_t batch_jobs = 0;
};

// Layout of one batch inside the arena: the batched workspace, then the
// gathered points, labels and core flags, then the small per-job arrays
// (offsets, eps, minPts, K, segments), which the host fills in one pinned
// mirror and copies with a single transfer.
struct BatchLayout {
  size_t ws = 0, ws_bytes = 0, pts = 0, lab = 0, core = 0, small = 0;
  size_t off = 0, eps = 0, mp = 0, ncl = 0, seg = 0, small_bytes = 0, total = 0;
};

bool batch_layout(int64_t n, int b, int dim, const fdb_options& o, BatchLayout* L) {
  size_t ws = 0;
  if (fdb_workspace_bytes_batched(n, b, dim, &o, &ws) != FDB_OK) return false;
  const size_t N = static_cast<size_t>(n), B = static_cast<size_t>(b);
  L->ws = 0;
  L->ws_bytes = ws;
  L->pts = align256(ws);
  L->lab = L->pts + align256(N * dim * 4);
  L->core = L->lab + align256(N * 4);
  L->small = L->core + align256(N);
  L->off = 0;
  L->eps = align256((B + 1) * 8);
  L->mp = L->eps + align256(B * 4);
  L->ncl = L->mp + align256(B * 4);
  L->seg = L->ncl + align256(B * 4);
  L->small_bytes = L->seg + align256(B * sizeof(JobSeg));
  L->total = L->small + L->small_bytes;
  return true;
}

size_t small_bytes_for(int b) {
  const size_t B = static_cast<size_t>(b);
  return align256((B + 1) * 8) + 3 * align256(B * 4) + align256(B * sizeof(JobSeg));
}

}  // namespace

namespace {

constexpr int kSlots = 2;  // batches that can be on the device at once (batched mode)

// One batch's place on the device: a share of the arena and everything a batch
// in flight needs of its own.
struct Slot {
  fdb_handle* h = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* arena = nullptr;
  size_t bytes = 0;
  char* host = nullptr;  // pinned mirror of the batch's small arrays; K and the info word come back here
  bool busy = false;
  std::vector<int64_t> ids;
  size_t ncl_off = 0, info_off = 0;
  int64_t t_launch = 0;
};

}  // namespace

struct fdb_server {
  int device = 0;
  int mode = FDB_SERVE_BATCHED;
  fdb_options opt{};
  size_t budget = 0;
  int max_batch = 1;
  std::vector<Slot> slots;
  char* arena = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::deque<Job> jobs;  // indexed by ticket; only appended to
  int64_t pending = 0;   // submitted and not yet done
  bool stop = false;
  int64_t batches = 0, max_queue = 0;
  int32_t max_batch_seen = 0;
  double busy_s = 0.0;    // time with at least one batch on the device
  int in_flight = 0;      // slots busy
  int64_t busy_since = 0;
  std::thread worker;
};

namespace {

void finish_jobs(fdb_server* s, const std::vector<int64_t>& ids, const std::vector<int32_t>& ncl,
                 const std::vector<int32_t>& st, int64_t t1) {
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t k = 0; k < ids.size(); ++k) {
    Job& j = s->jobs[ids[k]];
    j.num_clusters = ncl[k];
    j.status = st[k];
    j.t_done = t1;
    j.state = 2;
  }
  s->pending -= static_cast<int64_t>(ids.size());
  s->batches += 1;
  s->cv_done.notify_all();
}

// Start of a launch on the device / end of one (busy time is the union).
void mark_busy(fdb_server* s, int64_t t, int delta) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (delta > 0 && s->in_flight++ == 0) s->busy_since = t;
  if (delta < 0 && --s->in_flight == 0) s->busy_s += static_cast<double>(t - s->busy_since) * 1e-9;
}

// One batch into slot sl: gather, batched clustering, scatter, then K and the
// info word copied back and the slot's event recorded; nothing waits.
fdb_status launch_batch(fdb_server* s, Slot& sl, const std::vector<fdb_job>& in, int dim, int64_t n) {
  const int b = static_cast<int>(in.size());
  BatchLayout L;
  if (!batch_layout(n, b, dim, s->opt, &L) || L.total > sl.bytes) return FDB_ERR_NOMEM;
  char* small = sl.host;
  std::memset(small, 0, L.small_bytes);
  auto* off = reinterpret_cast<int64_t*>(small + L.off);
  auto* eps = reinterpret_cast<float*>(small + L.eps);
  auto* mp = reinterpret_cast<int32_t*>(small + L.mp);
  auto* seg = reinterpret_cast<JobSeg*>(small + L.seg);
  int64_t o = 0, gb = 0, sb = 0;
  for (int k = 0; k < b; ++k) {
    off[k] = o;
    eps[k] = in[k].eps;
    mp[k] = in[k].min_pts;
    seg[k].points = in[k].points;
    seg[k].labels = in[k].labels;
    seg[k].core = in[k].is_core;
    seg[k].n = in[k].n;
    seg[k].off = o;
    seg[k].gblk = static_cast<int32_t>(gb);
    seg[k].sblk = static_cast<int32_t>(sb);
    gb += fdb::seg_blocks(in[k].n * dim);
    sb += fdb::seg_blocks(in[k].n);
    o += in[k].n;
  }
  off[b] = o;
  char* base = sl.arena;
  char* dsmall = base + L.small;
  float* pts = reinterpret_cast<float*>(base + L.pts);
  int32_t* lab = reinterpret_cast<int32_t*>(base + L.lab);
  uint8_t* core = reinterpret_cast<uint8_t*>(base + L.core);
  const JobSeg* dseg = reinterpret_cast<const JobSeg*>(dsmall + L.seg);
  int32_t* dncl = reinterpret_cast<int32_t*>(dsmall + L.ncl);
  hipStream_t q = sl.stream;
  if (hipMemcpyAsync(dsmall, small, L.small_bytes, hipMemcpyHostToDevice, q) != hipSuccess) return FDB_ERR_HIP;
  fdb::launch_gather(dseg, b, gb, dim, pts, q);
  fdb_status r = fdb_dbscan_batched(sl.h, pts, n, reinterpret_cast<const int64_t*>(dsmall + L.off), b, dim,
                                    reinterpret_cast<const float*>(dsmall + L.eps),
                                    reinterpret_cast<const int32_t*>(dsmall + L.mp), &s->opt, lab, core, dncl,
                                    base + L.ws, L.ws_bytes, q);
  if (r != FDB_OK) return r;
  fdb::launch_scatter_jobs(dseg, b, sb, lab, core, q);
  // the mirror's small arrays were consumed by the copy above; K and the info word
  // land in their place (ordered after that copy on the stream)
  sl.ncl_off = L.ncl;
  sl.info_off = L.eps;
  if (hipMemcpyAsync(small + L.ncl, dncl, static_cast<size_t>(b) * 4, hipMemcpyDeviceToHost, q) != hipSuccess ||
      hipMemcpyAsync(small + L.eps, fdb::handle_info(sl.h), 4, hipMemcpyDeviceToHost, q) != hipSuccess ||
      hipEventRecord(sl.done, q) != hipSuccess)
    return FDB_ERR_HIP;
  return FDB_OK;
}

// A finished slot: its jobs' K and status from the pinned mirror.
void retire(fdb_server* s, Slot& sl, fdb_status r) {
  const size_t b = sl.ids.size();
  std::vector<int32_t> ncl(b, -1), st(b, static_cast<int32_t>(r));
  if (r == FDB_OK) {
    const int32_t* hncl = reinterpret_cast<const int32_t*>(sl.host + sl.ncl_off);
    const uint32_t info = *reinterpret_cast<const uint32_t*>(sl.host + sl.info_off);
    for (size_t k = 0; k < b; ++k) {
      ncl[k] = hncl[k];
      st[k] = (info & FDB_INFO_INTERNAL) ? FDB_ERR_INTERNAL : (hncl[k] < 0 ? FDB_ERR_NONFINITE : FDB_OK);
    }
  }
  const int64_t t = now_ns();
  finish_jobs(s, sl.ids, ncl, st, t);
  mark_busy(s, t, -1);
  sl.ids.clear();
  sl.busy = false;
}

// Takes the queued jobs of the oldest job's dim, in arrival order, while the
// batch fits in `bytes` and holds at most `cap` jobs (the first job always fits).
// Called with s->mu held.
int64_t take_batch(fdb_server* s, size_t bytes, int cap, std::vector<int64_t>& ids, std::vector<fdb_job>& in,
                   int* dim_out) {
  const int dim = s->jobs[s->queue.front()].in.dim;
  int64_t n = 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && static_cast<int>(ids.size()) < cap;) {
    const fdb_job& j = s->jobs[*it].in;
    if (j.dim != dim) {
      ++it;
      continue;
    }
    if (!ids.empty()) {
      BatchLayout L;
      if (!batch_layout(n + j.n, static_cast<int>(ids.size()) + 1, dim, s->opt, &L) || L.total > bytes) break;
    }
    ids.push_back(*it);
    in.push_back(j);
    n += j.n;
    it = s->queue.erase(it);
  }
  const int64_t t = now_ns();
  for (int64_t id : ids) {
    Job& j = s->jobs[id];
    j.state = 1;
    j.t_start = t;
    j.batch_jobs = static_cast<int32_t>(ids.size());
  }
  s->max_batch_seen = std::max(s->max_batch_seen, static_cast<int32_t>(ids.size()));
  *dim_out = dim;
  return n;
}

void worker_fifo(fdb_server* s) {
  Slot& sl = s->slots[0];
  std::vector<int64_t> ids;
  std::vector<fdb_job> in;
  for (;;) {
    ids.clear();
    in.clear();
    int dim = 3;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) return;  // stopping, and nothing left to run
      take_batch(s, sl.bytes, 1, ids, in, &dim);
    }
    const int64_t t0 = now_ns();
    mark_busy(s, t0, +1);
    const fdb_job& j = in[0];
    int32_t k = -1;
    fdb_status r = fdb_dbscan(sl.h, j.points, j.n, j.dim, j.eps, j.min_pts, &s->opt, j.labels, j.is_core, &k,
                              sl.arena, sl.bytes, sl.stream);
    if (r != FDB_OK && r != FDB_ERR_NONFINITE && r != FDB_ERR_INTERNAL) (void)hipStreamSynchronize(sl.stream);
    const int64_t t1 = now_ns();
    finish_jobs(s, ids, std::vector<int32_t>{k}, std::vector<int32_t>{static_cast<int32_t>(r)}, t1);
    mark_busy(s, t1, -1);
  }
}

void worker_batched(fdb_server* s) {
  std::vector<fdb_job> in;
  for (;;) {
    // hand back the slots whose batches have finished
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) continue;
      retire(s, sl, e == hipSuccess ? FDB_OK : FDB_ERR_HIP);
    }
    // fill the free slots with queued jobs
    bool launched = false;
    for (Slot& sl : s->slots) {
      if (sl.busy) continue;
      in.clear();
      int dim = 3;
      int64_t n = 0;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->queue.empty()) break;
        n = take_batch(s, sl.bytes, s->max_batch, sl.ids, in, &dim);
      }
      const int64_t t = now_ns();
      mark_busy(s, t, +1);
      sl.busy = true;
      sl.t_launch = t;
      const fdb_status r = launch_batch(s, sl, in, dim, n);
      if (r != FDB_OK) {
        (void)hipStreamSynchronize(sl.stream);
        retire(s, sl, r);
      }
      launched = true;
    }
    int busy = 0;
    Slot* oldest = nullptr;
    for (Slot& sl : s->slots)
      if (sl.busy) {
        ++busy;
        if (!oldest || sl.t_launch < oldest->t_launch) oldest = &sl;
      }
    if (launched) continue;
    if (busy == static_cast<int>(s->slots.size())) {
      (void)hipEventSynchronize(oldest->done);  // no slot free: nothing to do until one is
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (busy == 0) {
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) return;  // stopping, and nothing left to run
    } else if (s->queue.empty()) {
      // a batch runs and a slot is free: wake for a new job or poll the batch again
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

void worker_main(fdb_server* s) {
  (void)hipSetDevice(s->device);
  if (s->mode == FDB_SERVE_FIFO) worker_fifo(s);
  else worker_batched(s);
}

bool job_fits(const fdb_server* s, int64_t n, int dim) {
  const size_t bytes = s->slots[0].bytes;
  if (s->mode == FDB_SERVE_FIFO) {
    size_t ws = 0;
    return fdb_workspace_bytes(n, dim, &s->opt, &ws) == FDB_OK && ws <= bytes;
  }
  BatchLayout L;
  return batch_layout(n, 1, dim, s->opt, &L) && L.total <= bytes;
}

void fill_result(const Job& j, fdb_job_result* r) {
  r->done = j.state == 2 ? 1 : 0;
  r->status = j.state == 2 ? j.status : FDB_OK;
  r->num_clusters = j.state == 2 ? j.num_clusters : -1;
  r->batch_jobs = j.batch_jobs;
  r->queue_us = j.state >= 1 ? static_cast<double>(j.t_start - j.t_submit) * 1e-3 : -1.0;
  r->latency_us = j.state == 2 ? static_cast<double>(j.t_done - j.t_submit) * 1e-3 : -1.0;
}

// Frees what fdb_server_create set up (the device must be current).
void release(fdb_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h) fdb_destroy(sl.h);
  }
  s->slots.clear();
  if (s->arena) (void)hipFree(s->arena);
  s->arena = nullptr;
}

}  // namespace

extern "C" {

fdb_status fdb_server_create(int device, size_t hbm_budget_bytes, int32_t max_batch, int32_t mode,
                             const fdb_options* opt, fdb_server** out) {
  if (!out) return FDB_ERR_INVALID;
  *out = nullptr;
  fdb_options o{};
  if (opt) o = *opt;
  if ((mode != FDB_SERVE_BATCHED && mode != FDB_SERVE_FIFO) || max_batch < 1 || max_batch > (1 << 20) ||
      hbm_budget_bytes < (size_t(1) << 20))
    return FDB_ERR_INVALID;
  size_t probe = 0;
  if (fdb_workspace_bytes(0, 3, &o, &probe) != FDB_OK) return FDB_ERR_INVALID;  // validates the options
  fdb_server* s = new (std::nothrow) fdb_server;
  if (!s) return FDB_ERR_NOMEM;
  s->device = device;
  s->mode = mode;
  s->opt = o;
  s->budget = hbm_budget_bytes;
  s->max_batch = mode == FDB_SERVE_FIFO ? 1 : max_batch;
  const int nslots = mode == FDB_SERVE_FIFO ? 1 : kSlots;
  s->slots.resize(static_cast<size_t>(nslots));
  int prev = -1;
  (void)hipGetDevice(&prev);
  fdb_status r = FDB_OK;
  if (hipSetDevice(device) != hipSuccess) r = FDB_ERR_INVALID;
  if (r == FDB_OK && hipMalloc(reinterpret_cast<void**>(&s->arena), s->budget) != hipSuccess) r = FDB_ERR_NOMEM;
  const size_t share = s->budget / static_cast<size_t>(nslots) & ~size_t(255);
  for (int k = 0; k < nslots && r == FDB_OK; ++k) {
    Slot& sl = s->slots[static_cast<size_t>(k)];
    sl.arena = s->arena + share * static_cast<size_t>(k);
    sl.bytes = share;
    r = fdb_create(&sl.h, device);
    if (r == FDB_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) r = FDB_ERR_HIP;
    if (r == FDB_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) r = FDB_ERR_HIP;
    if (r == FDB_OK &&
        hipHostMalloc(reinterpret_cast<void**>(&sl.host), small_bytes_for(s->max_batch), hipHostMallocDefault) !=
            hipSuccess)
      r = FDB_ERR_NOMEM;
  }
  if (r == FDB_OK) {
    try {
      s->worker = std::thread(worker_main, s);
    } catch (...) {
      r = FDB_ERR_NOMEM;
    }
  }
  if (r != FDB_OK) release(s);
  if (prev >= 0) (void)hipSetDevice(prev);
  if (r != FDB_OK) {
    delete s;
    return r;
  }
  *out = s;
  return FDB_OK;
}

fdb_status fdb_server_submit(fdb_server* s, const fdb_job* job, int64_t* h_ticket) {
  if (!s || !job || !h_ticket) return FDB_ERR_INVALID;
  const fdb_job& j = *job;
  if ((j.dim != 2 && j.dim != 3) || j.n < 0 || j.n > fdb::kMaxPoints || !std::isfinite(j.eps) || !(j.eps > 0.0f) ||
      j.min_pts < 1)
    return FDB_ERR_INVALID;
  if (j.n > 0 && (!j.points || !j.labels)) return FDB_ERR_INVALID;
  if (!job_fits(s, j.n, j.dim)) return FDB_ERR_NOMEM;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return FDB_ERR_INVALID;
    const int64_t ticket = static_cast<int64_t>(s->jobs.size());
    s->jobs.emplace_back();
    Job& rec = s->jobs.back();
    rec.in = j;
    rec.t_submit = now_ns();
    if (j.n == 0) {
      rec.state = 2;
      rec.t_start = rec.t_done = rec.t_submit;
      s->cv_done.notify_all();
    } else {
      s->queue.push_back(ticket);
      s->pending += 1;
      s->max_queue = std::max(s->max_queue, static_cast<int64_t>(s->queue.size()));
    }
    *h_ticket = ticket;
  }
  s->cv_work.notify_one();
  return FDB_OK;
}

fdb_status fdb_server_poll(fdb_server* s, int64_t ticket, fdb_job_result* h_out) {
  if (!s || !h_out) return FDB_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket < 0 || ticket >= static_cast<int64_t>(s->jobs.size())) return FDB_ERR_INVALID;
  fill_result(s->jobs[ticket], h_out);
  return FDB_OK;
}

fdb_status fdb_server_wait(fdb_server* s, int64_t ticket, fdb_job_result* h_out) {
  if (!s) return FDB_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket < 0 || ticket >= static_cast<int64_t>(s->jobs.size())) return FDB_ERR_INVALID;
  s->cv_done.wait(lk, [&] { return s->jobs[ticket].state == 2; });
  if (h_out) fill_result(s->jobs[ticket], h_out);
  return FDB_OK;
}

fdb_status fdb_server_drain(fdb_server* s) {
  if (!s) return FDB_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending == 0; });
  return FDB_OK;
}

fdb_status fdb_server_stats(fdb_server* s, int64_t first_ticket, fdb_serve_stats* h_out) {
  if (!s || !h_out || first_ticket < 0) return FDB_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(h_out, 0, sizeof(*h_out));
  std::vector<double> lat;
  int64_t t_first = 0, t_last = 0;
  for (int64_t t = first_ticket; t < static_cast<int64_t>(s->jobs.size()); ++t) {
    const Job& j = s->jobs[t];
    if (j.state != 2 || j.in.n == 0) continue;
    lat.push_back(static_cast<double>(j.t_done - j.t_submit) * 1e-3);
    h_out->points += j.in.n;
    if (lat.size() == 1 || j.t_submit < t_first) t_first = j.t_submit;
    t_last = std::max(t_last, j.t_done);
  }
  h_out->jobs = static_cast<int64_t>(lat.size());
  h_out->batches = s->batches;
  h_out->busy_s = s->busy_s;
  h_out->max_queue = s->max_queue;
  h_out->max_batch_jobs = s->max_batch_seen;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto rank = [&](double q) {  // nearest-rank percentile
      size_t k = static_cast<size_t>(std::ceil(q * static_cast<double>(lat.size())));
      return lat[std::min(lat.size(), std::max<size_t>(k, 1)) - 1];
    };
    double sum = 0.0;
    for (double v : lat) sum += v;
    h_out->p50_us = rank(0.50);
    h_out->p99_us = rank(0.99);
    h_out->mean_us = sum / static_cast<double>(lat.size());
    h_out->max_us = lat.back();
    h_out->span_s = static_cast<double>(t_last - t_first) * 1e-9;
  }
  return FDB_OK;
}

void fdb_server_destroy(fdb_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  release(s);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
