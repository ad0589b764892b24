"""CPU oracle for DBSCAN - test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU library never links, loads or calls it, and this package
never imports the GPU library.

`oracle.c` computes the DBSCAN definition of Section 2.1 of the paper (core
points, connected components of the core graph, border and noise points) with
the canonical output encoding described in its header. This module loads the
compiled C code with ctypes and wraps it for numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.oracle_pred.argtypes = [fp, fp, ctypes.c_int, ctypes.c_float]
        lib.oracle_pred.restype = ctypes.c_int
        lib.oracle_eps2.argtypes = [ctypes.c_float]
        lib.oracle_eps2.restype = ctypes.c_float
        lib.oracle_neighbor_counts.argtypes = [fp, ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                                               ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_neighbor_counts.restype = ctypes.c_int
        lib.oracle_dbscan.argtypes = [fp, ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_int32,
                                      ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_dbscan.restype = ctypes.c_int64
        lib.oracle_check_border.argtypes = [fp, ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.c_int, ctypes.c_int]
        lib.oracle_check_border.restype = ctypes.c_int64
        lib.oracle_neighbors_of.argtypes = [fp, ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
        lib.oracle_neighbors_of.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _as_points(points) -> np.ndarray:
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32))
    if pts.ndim != 2 or pts.shape[1] not in (2, 3):
        raise ValueError("points must be [n, 2] or [n, 3]")
    return pts


def _mode(method: str, n: int) -> int:
    if method == "auto":
        return 0 if n <= 4096 else 1
    return {"brute": 0, "grid": 1}[method]


def pred(p, q, eps: float) -> bool:
    """The fp32 neighbour test for one pair of points."""
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float32))
    lib = _load()
    fp = ctypes.POINTER(ctypes.c_float)
    e2 = lib.oracle_eps2(ctypes.c_float(eps))
    return bool(lib.oracle_pred(p.ctypes.data_as(fp), q.ctypes.data_as(fp), int(p.shape[0]), e2))


def neighbor_counts(points, eps: float, method: str = "auto", threads: int = 0) -> np.ndarray:
    """|N_eps(x)| for every point, x itself included."""
    pts = _as_points(points)
    n, d = pts.shape
    out = np.zeros(n, dtype=np.int32)
    rc = _load().oracle_neighbor_counts(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, d,
                                        ctypes.c_float(eps), _mode(method, n), threads,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise RuntimeError(f"oracle_neighbor_counts failed ({rc})")
    return out


def dbscan(points, eps: float, min_pts: int, method: str = "auto", threads: int = 0):
    """Canonical DBSCAN labels.

    Returns (labels int32 [n], is_core bool [n], K). labels: -1 noise, else the
    cluster id 0..K-1, ordered by the smallest input index among each cluster's
    core points; a border point takes the smallest id among the clusters that
    hold a core point within eps of it.
    """
    pts = _as_points(points)
    n, d = pts.shape
    labels = np.empty(n, dtype=np.int32)
    core = np.empty(n, dtype=np.uint8)
    k = _load().oracle_dbscan(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, d,
                              ctypes.c_float(eps), int(min_pts), _mode(method, n), threads,
                              labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              core.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if k < 0:
        raise RuntimeError(f"oracle_dbscan failed ({k})")
    return labels, core.astype(bool), int(k)


def dbscan_star(points, eps: float, min_pts: int, method: str = "auto", threads: int = 0):
    """DBSCAN* (Section 2.1): the clusters are the connected components of the
    core points, and every non-core point is noise. Cluster ids are the
    canonical ones (they depend on core points only)."""
    labels, core, k = dbscan(points, eps, min_pts, method, threads)
    labels = np.where(core, labels, -1).astype(np.int32)
    return labels, core, k


def check_border(points, eps: float, is_core, labels, method: str = "auto", threads: int = 0) -> int:
    """Number of non-core points whose label breaks the definition: a labelled
    non-core point needs a same-label core within eps; a noise point needs none."""
    pts = _as_points(points)
    n, d = pts.shape
    core = np.ascontiguousarray(np.asarray(is_core, dtype=np.uint8))
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    bad = _load().oracle_check_border(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, d,
                                      ctypes.c_float(eps),
                                      core.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                      lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      _mode(method, n), threads)
    if bad < 0:
        raise RuntimeError(f"oracle_check_border failed ({bad})")
    return int(bad)


def neighbors_of(points, eps: float, i: int, cap: int = 1 << 20) -> np.ndarray:
    """Indices j (increasing) with point i within eps of point j, by brute force over all points."""
    pts = _as_points(points)
    n, d = pts.shape
    out = np.empty(cap, dtype=np.int64)
    k = _load().oracle_neighbors_of(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, d, ctypes.c_float(eps),
                                    int(i), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap)
    if k < 0:
        raise RuntimeError("oracle_neighbors_of failed")
    if k > cap:
        return neighbors_of(points, eps, i, cap=int(k))
    return out[:k].copy()
