"""ctypes binding of libfdbscan (include/fdbscan.h): argument marshalling only.

Every step of the clustering runs in the library's HIP kernels; PyTorch only
provides device memory and the stream. The library is loaded from this
directory; if it has not been built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdbscan.so")

(FDB_OK, FDB_ERR_INVALID, FDB_ERR_NOMEM, FDB_ERR_HIP, FDB_ERR_NONFINITE, FDB_ERR_INTERNAL, FDB_ERR_BUSY,
 FDB_ERR_SCRATCH) = range(8)
FDB_NOALLOC_SCRATCH_BYTES = 64 << 20
FDB_ALGO_FDBSCAN, FDB_ALGO_DENSEBOX, FDB_ALGO_AUTO = 0, 1, 2
FDB_BORDER_CANONICAL, FDB_BORDER_FIRST, FDB_BORDER_NONE = 0, 1, 2
FDB_INFO_DENSEBOX_FALLBACK, FDB_INFO_NONFINITE, FDB_INFO_INTERNAL, FDB_INFO_BAD_PARAMS = 1, 2, 4, 8
FDB_INFO_AUTO_FDBSCAN = 16
FDB_INFO_FOREST = 32
FDB_FLAG_GRAPH, FDB_FLAG_VALIDATE = 1, 2

ALGOS = {"fdbscan": FDB_ALGO_FDBSCAN, "densebox": FDB_ALGO_DENSEBOX, "auto": FDB_ALGO_AUTO}
BORDERS = {"canonical": FDB_BORDER_CANONICAL, "first": FDB_BORDER_FIRST, "none": FDB_BORDER_NONE}


class FdbOptions(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("border", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("tile", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FdbJob(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("eps", ctypes.c_float),
                ("min_pts", ctypes.c_int32), ("labels", ctypes.c_void_p), ("is_core", ctypes.c_void_p)]


class FdbJobResult(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("num_clusters", ctypes.c_int32),
                ("batch_jobs", ctypes.c_int32), ("queue_us", ctypes.c_double), ("latency_us", ctypes.c_double)]


class FdbServeStats(ctypes.Structure):
    _fields_ = [("jobs", ctypes.c_int64), ("points", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_queue", ctypes.c_int64), ("max_batch_jobs", ctypes.c_int32), ("span_s", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double)]


FDB_SERVE_BATCHED, FDB_SERVE_FIFO = 0, 1
SERVE_MODES = {"batched": FDB_SERVE_BATCHED, "fifo": FDB_SERVE_FIFO}


class FdbError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libfdbscan.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with __graft_entry__.build() "
                           "or python paper_2103_05162_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.fdb_status_string.argtypes = [ctypes.c_int]
    lib.fdb_status_string.restype = ctypes.c_char_p
    lib.fdb_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.fdb_create.restype = ctypes.c_int
    lib.fdb_destroy.argtypes = [vp]
    lib.fdb_destroy.restype = None
    lib.fdb_workspace_bytes.argtypes = [i64, i32, ctypes.POINTER(FdbOptions), ctypes.POINTER(sz)]
    lib.fdb_workspace_bytes.restype = ctypes.c_int
    lib.fdb_dbscan.argtypes = [vp, vp, i64, i32, ctypes.c_float, i32, ctypes.POINTER(FdbOptions), vp, vp,
                               ctypes.POINTER(i32), vp, sz, vp]
    lib.fdb_dbscan.restype = ctypes.c_int
    lib.fdb_dbscan_noalloc.argtypes = [vp, vp, i64, i32, ctypes.c_float, i32, ctypes.POINTER(FdbOptions), vp, vp,
                                       ctypes.POINTER(i32), vp]
    lib.fdb_dbscan_noalloc.restype = ctypes.c_int
    lib.fdb_workspace_bytes_batched.argtypes = [i64, i32, i32, ctypes.POINTER(FdbOptions), ctypes.POINTER(sz)]
    lib.fdb_workspace_bytes_batched.restype = ctypes.c_int
    lib.fdb_dbscan_batched.argtypes = [vp, vp, i64, vp, i32, i32, vp, vp, ctypes.POINTER(FdbOptions), vp, vp, vp, vp,
                                       sz, vp]
    lib.fdb_dbscan_batched.restype = ctypes.c_int
    lib.fdb_dbscan_batched_host.argtypes = [vp, vp, vp, i32, i32, vp, vp, ctypes.POINTER(FdbOptions), sz, vp, vp,
                                            vp]
    lib.fdb_dbscan_batched_host.restype = ctypes.c_int
    lib.fdb_last_info.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
    lib.fdb_last_info.restype = ctypes.c_int
    lib.fdb_last_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint32)]
    lib.fdb_last_status.restype = ctypes.c_int
    po, pd = ctypes.POINTER(FdbOptions), ctypes.POINTER(ctypes.c_double)
    lib.fdb_tune.argtypes = [vp, vp, i64, i32, ctypes.c_float, i32, po, i32, vp, vp, vp, sz, vp, po, pd]
    lib.fdb_tune.restype = ctypes.c_int
    lib.fdb_tune_batched.argtypes = [vp, vp, i64, vp, i32, i32, vp, vp, po, i32, vp, vp, vp, vp, sz, vp, po, pd]
    lib.fdb_tune_batched.restype = ctypes.c_int
    lib.fdb_tuned_options.argtypes = [vp, i64, i32, i32, i32, po, po]
    lib.fdb_tuned_options.restype = ctypes.c_int
    lib.fdb_last_counts.argtypes = [vp, ctypes.POINTER(i64)]
    lib.fdb_last_counts.restype = ctypes.c_int
    pi32 = ctypes.POINTER(i32)
    lib.fdb_debug_forest.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64)]
    lib.fdb_debug_forest.restype = ctypes.c_int
    lib.fdb_debug_lbvh.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32, i32, i32, pi32, pi32, pi32, pi32]
    lib.fdb_debug_lbvh.restype = ctypes.c_int
    lib.fdb_set_timing.argtypes = [vp, i32]
    lib.fdb_set_timing.restype = ctypes.c_int
    lib.fdb_stage_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fdb_stage_times.restype = ctypes.c_int
    lib.fdb_server_create.argtypes = [ctypes.c_int, sz, i32, i32, ctypes.POINTER(FdbOptions), ctypes.POINTER(vp)]
    lib.fdb_server_create.restype = ctypes.c_int
    lib.fdb_server_submit.argtypes = [vp, ctypes.POINTER(FdbJob), ctypes.POINTER(i64)]
    lib.fdb_server_submit.restype = ctypes.c_int
    lib.fdb_server_poll.argtypes = [vp, i64, ctypes.POINTER(FdbJobResult)]
    lib.fdb_server_poll.restype = ctypes.c_int
    lib.fdb_server_wait.argtypes = [vp, i64, ctypes.POINTER(FdbJobResult)]
    lib.fdb_server_wait.restype = ctypes.c_int
    lib.fdb_server_drain.argtypes = [vp]
    lib.fdb_server_drain.restype = ctypes.c_int
    lib.fdb_server_stats.argtypes = [vp, i64, ctypes.POINTER(FdbServeStats)]
    lib.fdb_server_stats.restype = ctypes.c_int
    lib.fdb_server_destroy.argtypes = [vp]
    lib.fdb_server_destroy.restype = None
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().fdb_status_string(int(status)).decode()


def _check(status: int, what: str) -> None:
    if status != FDB_OK:
        raise FdbError(status, what)


def make_options(algo="fdbscan", border="canonical", leaf_size=0, block_size=0, flags=0, tile=0,
                 graph=False, validate=False) -> FdbOptions:
    a = ALGOS[algo] if isinstance(algo, str) else int(algo)
    b = BORDERS[border] if isinstance(border, str) else int(border)
    f = int(flags) | (FDB_FLAG_GRAPH if graph else 0) | (FDB_FLAG_VALIDATE if validate else 0)
    return FdbOptions(a, b, int(leaf_size), int(block_size), int(tile), f)


def options_dict(o: FdbOptions) -> dict:
    return {k: int(getattr(o, k)) for k, _ in FdbOptions._fields_}


def workspace_bytes_batched(n_total: int, num_clouds: int, dim: int, algo="fdbscan") -> int:
    out = ctypes.c_size_t(0)
    opt = make_options(algo)
    _check(load().fdb_workspace_bytes_batched(int(n_total), int(num_clouds), int(dim), ctypes.byref(opt),
                                              ctypes.byref(out)), "fdb_workspace_bytes_batched")
    return int(out.value)


def workspace_bytes(n: int, dim: int, algo="fdbscan") -> int:
    out = ctypes.c_size_t(0)
    opt = make_options(algo)
    _check(load().fdb_workspace_bytes(int(n), int(dim), ctypes.byref(opt), ctypes.byref(out)), "fdb_workspace_bytes")
    return int(out.value)


class Handle:
    """An fdb_handle bound to one HIP device (owns a cached workspace)."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.fdb_create(ctypes.byref(h), int(device)), "fdb_create")
        self.ptr = h
        self.device = int(device)

    def close(self) -> None:
        if getattr(self, "ptr", None):
            self._lib.fdb_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dbscan_raw(self, points_ptr: int, n: int, dim: int, eps: float, min_pts: int, labels_ptr: int,
                   core_ptr: int | None, stream: int, options: FdbOptions | None = None, want_k: bool = True,
                   workspace_ptr: int | None = None, workspace_size: int = 0):
        """fdb_dbscan on raw device pointers. Returns K (or None when want_k is False)."""
        k = ctypes.c_int32(-1)
        st = self._lib.fdb_dbscan(self.ptr, ctypes.c_void_p(points_ptr), int(n), int(dim), ctypes.c_float(eps),
                                  int(min_pts), ctypes.byref(options) if options is not None else None,
                                  ctypes.c_void_p(labels_ptr), ctypes.c_void_p(core_ptr) if core_ptr else None,
                                  ctypes.byref(k) if want_k else None,
                                  ctypes.c_void_p(workspace_ptr) if workspace_ptr else None, int(workspace_size),
                                  ctypes.c_void_p(stream))
        _check(st, "fdb_dbscan")
        return int(k.value) if want_k else None

    def dbscan_noalloc_raw(self, points_ptr: int, n: int, dim: int, eps: float, min_pts: int, labels_ptr: int,
                           core_ptr: int | None, stream: int, options: FdbOptions | None = None,
                           want_k: bool = True):
        """fdb_dbscan_noalloc on raw device pointers. Returns K (or None when want_k is False)."""
        k = ctypes.c_int32(-1)
        st = self._lib.fdb_dbscan_noalloc(self.ptr, ctypes.c_void_p(points_ptr), int(n), int(dim),
                                          ctypes.c_float(eps), int(min_pts),
                                          ctypes.byref(options) if options is not None else None,
                                          ctypes.c_void_p(labels_ptr), ctypes.c_void_p(core_ptr) if core_ptr else None,
                                          ctypes.byref(k) if want_k else None, ctypes.c_void_p(stream))
        _check(st, "fdb_dbscan_noalloc")
        return int(k.value) if want_k else None

    def dbscan_batched_raw(self, points_ptr: int, n_total: int, offsets_ptr: int, num_clouds: int, dim: int,
                           eps_ptr: int, min_pts_ptr: int, labels_ptr: int, core_ptr: int | None,
                           num_clusters_ptr: int | None, stream: int, options: FdbOptions | None = None,
                           workspace_ptr: int | None = None, workspace_size: int = 0) -> None:
        """fdb_dbscan_batched on raw device pointers (asynchronous)."""
        vp = ctypes.c_void_p
        st = self._lib.fdb_dbscan_batched(self.ptr, vp(points_ptr), int(n_total), vp(offsets_ptr), int(num_clouds),
                                          int(dim), vp(eps_ptr), vp(min_pts_ptr),
                                          ctypes.byref(options) if options is not None else None, vp(labels_ptr),
                                          vp(core_ptr) if core_ptr else None,
                                          vp(num_clusters_ptr) if num_clusters_ptr else None,
                                          vp(workspace_ptr) if workspace_ptr else None, int(workspace_size), vp(stream))
        _check(st, "fdb_dbscan_batched")

    def dbscan_batched_host_raw(self, points_ptr: int, offsets_ptr: int, num_clouds: int, dim: int, eps_ptr: int,
                                min_pts_ptr: int, budget_bytes: int, labels_ptr: int, core_ptr: int | None,
                                num_clusters_ptr: int, options: FdbOptions | None = None) -> None:
        """fdb_dbscan_batched_host on raw host pointers (synchronous)."""
        vp = ctypes.c_void_p
        st = self._lib.fdb_dbscan_batched_host(self.ptr, vp(points_ptr) if points_ptr else None, vp(offsets_ptr),
                                               int(num_clouds), int(dim), vp(eps_ptr), vp(min_pts_ptr),
                                               ctypes.byref(options) if options is not None else None,
                                               int(budget_bytes), vp(labels_ptr) if labels_ptr else None,
                                               vp(core_ptr) if core_ptr else None, vp(num_clusters_ptr))
        _check(st, "fdb_dbscan_batched_host")

    def last_info(self) -> int:
        v = ctypes.c_uint32(0)
        _check(self._lib.fdb_last_info(self.ptr, ctypes.byref(v)), "fdb_last_info")
        return int(v.value)

    def last_status(self, stream: int):
        """(status, FDB_INFO_* bits) of the last call, waiting for `stream`."""
        v = ctypes.c_uint32(0)
        st = self._lib.fdb_last_status(self.ptr, ctypes.c_void_p(stream), ctypes.byref(v))
        return int(st), int(v.value)

    def tune_raw(self, points_ptr: int, n: int, dim: int, eps: float, min_pts: int, labels_ptr: int,
                 core_ptr: int | None, stream: int, options: FdbOptions | None = None, reps: int = 3,
                 workspace_ptr: int | None = None, workspace_size: int = 0):
        """fdb_tune: returns (best options, best ms, default ms)."""
        best = FdbOptions()
        ms = (ctypes.c_double * 2)()
        vp = ctypes.c_void_p
        st = self._lib.fdb_tune(self.ptr, vp(points_ptr), int(n), int(dim), ctypes.c_float(eps), int(min_pts),
                                ctypes.byref(options) if options is not None else None, int(reps), vp(labels_ptr),
                                vp(core_ptr) if core_ptr else None, vp(workspace_ptr) if workspace_ptr else None,
                                int(workspace_size), vp(stream), ctypes.byref(best), ms)
        _check(st, "fdb_tune")
        return best, float(ms[0]), float(ms[1])

    def tune_batched_raw(self, points_ptr: int, n_total: int, offsets_ptr: int, num_clouds: int, dim: int,
                         eps_ptr: int, min_pts_ptr: int, labels_ptr: int, core_ptr: int | None,
                         num_clusters_ptr: int | None, stream: int, options: FdbOptions | None = None, reps: int = 3,
                         workspace_ptr: int | None = None, workspace_size: int = 0):
        """fdb_tune_batched: returns (best options, best ms, default ms)."""
        best = FdbOptions()
        ms = (ctypes.c_double * 2)()
        vp = ctypes.c_void_p
        st = self._lib.fdb_tune_batched(self.ptr, vp(points_ptr), int(n_total), vp(offsets_ptr), int(num_clouds),
                                        int(dim), vp(eps_ptr), vp(min_pts_ptr),
                                        ctypes.byref(options) if options is not None else None, int(reps),
                                        vp(labels_ptr), vp(core_ptr) if core_ptr else None,
                                        vp(num_clusters_ptr) if num_clusters_ptr else None,
                                        vp(workspace_ptr) if workspace_ptr else None, int(workspace_size),
                                        vp(stream), ctypes.byref(best), ms)
        _check(st, "fdb_tune_batched")
        return best, float(ms[0]), float(ms[1])

    def tuned_options(self, n: int, dim: int, min_pts: int, num_clouds: int = 0,
                      options: FdbOptions | None = None) -> FdbOptions:
        out = FdbOptions()
        _check(self._lib.fdb_tuned_options(self.ptr, int(n), int(dim), int(min_pts), int(num_clouds),
                                           ctypes.byref(options) if options is not None else None,
                                           ctypes.byref(out)), "fdb_tuned_options")
        return out

    def last_counts(self) -> dict:
        """Sizes of the last call: clusters, grid cells, dense cells, BVH primitives."""
        v = (ctypes.c_int64 * 4)()
        _check(self._lib.fdb_last_counts(self.ptr, v), "fdb_last_counts")
        return {"clusters": int(v[0]), "cells": int(v[1]), "dense_cells": int(v[2]), "prims": int(v[3])}

    def debug_forest(self, parent_ptr: int, core_ptr: int | None, n: int) -> int:
        """Test hook: points of the forest parent[n] that break the main phase's invariants."""
        bad = ctypes.c_int64(-1)
        _check(self._lib.fdb_debug_forest(self.ptr, ctypes.c_void_p(parent_ptr),
                                          ctypes.c_void_p(core_ptr) if core_ptr else None, int(n),
                                          ctypes.byref(bad)), "fdb_debug_forest")
        return int(bad.value)

    def debug_lbvh(self, keys, mask: int = -1, leaf_size: int = 1):
        """Test hook: (gamma, other, leaves reached by a walk masked at `mask`) for sorted keys."""
        import numpy as np
        k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
        m = int(k.size)
        gamma = np.zeros(max(m - 1, 1), np.int32)
        other = np.zeros(max(m - 1, 1), np.int32)
        leaves = np.zeros(m, np.int32)
        cnt = ctypes.c_int32(0)
        p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        _check(self._lib.fdb_debug_lbvh(self.ptr, k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), m, int(mask),
                                        int(leaf_size), p(gamma), p(other), p(leaves), ctypes.byref(cnt)),
               "fdb_debug_lbvh")
        return gamma[:m - 1], other[:m - 1], leaves[:min(cnt.value, m)]

    def set_timing(self, enable: bool) -> None:
        _check(self._lib.fdb_set_timing(self.ptr, 1 if enable else 0), "fdb_set_timing")

    def stage_times(self):
        """(dict stage -> total ms, number of timed calls)."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32(0)
        calls = ctypes.c_int32(0)
        _check(self._lib.fdb_stage_times(self.ptr, cap, names, ms, ctypes.byref(cnt), ctypes.byref(calls)),
               "fdb_stage_times")
        return {names[i].decode(): ms[i] for i in range(min(cnt.value, cap))}, int(calls.value)


def _result(r: FdbJobResult) -> dict:
    return {"done": bool(r.done), "status": int(r.status), "num_clusters": int(r.num_clusters),
            "batch_jobs": int(r.batch_jobs), "queue_us": float(r.queue_us), "latency_us": float(r.latency_us)}


class Server:
    """fdb_server: a job queue served by continuous batching ("batched") or one job
    at a time ("fifo") inside a fixed device-memory budget."""

    def __init__(self, device: int = 0, budget_bytes: int = 8 << 30, max_batch: int = 4096, mode: str = "batched",
                 algo="fdbscan", border="canonical"):
        self._lib = load()
        p = ctypes.c_void_p()
        opt = make_options(algo, border)
        _check(self._lib.fdb_server_create(int(device), int(budget_bytes), int(max_batch), SERVE_MODES[mode],
                                           ctypes.byref(opt), ctypes.byref(p)), "fdb_server_create")
        self.ptr = p

    def submit_raw(self, points_ptr: int, n: int, dim: int, eps: float, min_pts: int, labels_ptr: int,
                   core_ptr: int | None = None) -> int:
        job = FdbJob(ctypes.c_void_p(points_ptr or None), int(n), int(dim), ctypes.c_float(eps), int(min_pts),
                     ctypes.c_void_p(labels_ptr or None), ctypes.c_void_p(core_ptr) if core_ptr else None)
        t = ctypes.c_int64(-1)
        _check(self._lib.fdb_server_submit(self.ptr, ctypes.byref(job), ctypes.byref(t)), "fdb_server_submit")
        return int(t.value)

    def poll(self, ticket: int) -> dict:
        r = FdbJobResult()
        _check(self._lib.fdb_server_poll(self.ptr, int(ticket), ctypes.byref(r)), "fdb_server_poll")
        return _result(r)

    def wait(self, ticket: int) -> dict:
        r = FdbJobResult()
        _check(self._lib.fdb_server_wait(self.ptr, int(ticket), ctypes.byref(r)), "fdb_server_wait")
        return _result(r)

    def drain(self) -> None:
        _check(self._lib.fdb_server_drain(self.ptr), "fdb_server_drain")

    def stats(self, first_ticket: int = 0) -> dict:
        st = FdbServeStats()
        _check(self._lib.fdb_server_stats(self.ptr, int(first_ticket), ctypes.byref(st)), "fdb_server_stats")
        return {k: getattr(st, k) for k, _ in FdbServeStats._fields_}

    def close(self) -> None:
        if getattr(self, "ptr", None):
            self._lib.fdb_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
