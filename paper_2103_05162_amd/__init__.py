"""Tree-based DBSCAN (FDbscan and FDbscan-DenseBox) for 2D/3D float32 points on
AMD Instinct MI355X, after Prokopenko, Lebrun-Grandie and Arndt, "Fast
tree-based algorithms for DBSCAN for low-dimensional data on GPUs" (ICPP 2023).

The clustering runs entirely in libfdbscan's HIP kernels (C ABI in
include/fdbscan.h); this package marshals torch tensors into that ABI.
"""
from __future__ import annotations

from ._lib import (FDB_ERR_BUSY, FDB_ERR_SCRATCH, FDB_FLAG_GRAPH, FDB_FLAG_VALIDATE, FDB_INFO_FOREST,
                   FDB_NOALLOC_SCRATCH_BYTES, FDB_INFO_AUTO_FDBSCAN, FDB_INFO_BAD_PARAMS,
                   FDB_INFO_DENSEBOX_FALLBACK, FDB_INFO_INTERNAL, FDB_INFO_NONFINITE, FdbError, Handle, Server, load,
                   make_options, options_dict, status_string, workspace_bytes, workspace_bytes_batched)

__all__ = ["dbscan", "dbscan_noalloc", "dbscan_batched", "dbscan_batched_host", "tune", "tune_batched", "Handle", "Server", "FdbError",
           "workspace_bytes", "workspace_bytes_batched", "default_handle", "load", "make_options", "options_dict",
           "status_string", "FDB_INFO_DENSEBOX_FALLBACK", "FDB_INFO_NONFINITE", "FDB_INFO_INTERNAL",
           "FDB_INFO_BAD_PARAMS", "FDB_INFO_AUTO_FDBSCAN", "FDB_FLAG_GRAPH", "FDB_ERR_BUSY", "FDB_ERR_SCRATCH",
           "FDB_NOALLOC_SCRATCH_BYTES", "FDB_FLAG_VALIDATE", "FDB_INFO_FOREST"]

_handles: dict[int, Handle] = {}


def default_handle(device: int = 0) -> Handle:
    h = _handles.get(device)
    if h is None:
        h = Handle(device)
        _handles[device] = h
    return h


def _check_out(labels, is_core, n):
    """Caller-supplied outputs: int32 labels and one byte (uint8 or bool) per core flag, n of each, contiguous."""
    import torch
    if labels.dtype != torch.int32 or labels.numel() < n or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous int32 tensor of at least n elements")
    if is_core.dtype not in (torch.uint8, torch.bool) or is_core.numel() < n or not is_core.is_contiguous():
        raise ValueError("is_core must be a contiguous uint8 or bool tensor of at least n elements")


def dbscan(points, eps: float, min_pts: int, algo: str = "fdbscan", border: str = "canonical",
           leaf_size: int = 0, block_size: int = 0, handle: Handle | None = None, labels=None, is_core=None,
           want_k: bool = True, workspace=None, tile: int = 0, graph: bool = False, validate: bool = False):
    """Cluster points ([n, 2] or [n, 3] float32 torch tensor on a HIP device).

    Returns (labels int32 [n], is_core bool [n], K). labels are in input order:
    -1 noise, else a cluster id 0..K-1 (canonical order unless border="first";
    border="none" is DBSCAN*: every non-core point is noise).
    K is None when want_k is False (then the call does not wait for the GPU).
    graph=True replays a recorded HIP graph of the launch sequence for repeated
    calls with the same buffers and parameters. validate=True checks the
    union-find forest after the main phase (FDB_INFO_FOREST on a violation).
    """
    import torch

    if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
        raise TypeError("points must be a torch tensor on a HIP device")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] not in (2, 3):
        raise ValueError("points must be float32 with shape [n, 2] or [n, 3]")
    pts = points.contiguous()
    n, d = pts.shape
    dev = pts.device.index if pts.device.index is not None else torch.cuda.current_device()
    h = handle if handle is not None else default_handle(dev)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=pts.device)
    if is_core is None:
        is_core = torch.empty(n, dtype=torch.uint8, device=pts.device)
    _check_out(labels, is_core, n)
    opt = make_options(algo, border, leaf_size, block_size, tile=tile, graph=graph, validate=validate)
    stream = torch.cuda.current_stream(pts.device).cuda_stream
    ws_ptr, ws_size = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    k = h.dbscan_raw(pts.data_ptr() if n else 0, n, d, eps, min_pts, labels.data_ptr() if n else 0,
                     is_core.data_ptr() if n else 0, stream, opt, want_k, ws_ptr, ws_size)
    return labels, is_core.view(torch.bool), k


def dbscan_noalloc(points, eps: float, min_pts: int, labels, is_core, algo: str = "fdbscan",
                   border: str = "canonical", leaf_size: int = 0, block_size: int = 0, tile: int = 0,
                   handle: Handle | None = None, want_k: bool = True):
    """fdb_dbscan_noalloc: dbscan() in the library's static scratch, with caller-owned
    outputs (labels int32 [n], is_core uint8 [n]); nothing is allocated. Returns K
    (None when want_k is False)."""
    import torch

    if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
        raise TypeError("points must be a torch tensor on a HIP device")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] not in (2, 3) \
            or not points.is_contiguous():
        raise ValueError("points must be contiguous float32 with shape [n, 2] or [n, 3]")
    n, d = points.shape
    _check_out(labels, is_core, n)
    dev = points.device.index if points.device.index is not None else torch.cuda.current_device()
    h = handle if handle is not None else default_handle(dev)
    opt = make_options(algo, border, leaf_size, block_size, tile=tile)
    stream = torch.cuda.current_stream(points.device).cuda_stream
    return h.dbscan_noalloc_raw(points.data_ptr() if n else 0, n, d, eps, min_pts, labels.data_ptr() if n else 0,
                                is_core.data_ptr() if n else 0, stream, opt, want_k)


def dbscan_batched(points, offsets, eps, min_pts, algo: str = "fdbscan", border: str = "canonical",
                   leaf_size: int = 0, block_size: int = 0, handle: Handle | None = None, labels=None, is_core=None,
                   num_clusters=None, workspace=None, tile: int = 0, graph: bool = False, validate: bool = False):
    """Cluster a batch of clouds in one launch sequence.

    points: [N, d] float32 on a HIP device (clouds concatenated); offsets: int64
    [B+1] (cloud c = points[offsets[c]:offsets[c+1]]); eps: float32 [B];
    min_pts: int32 [B] (all on the same device). Returns (labels int32 [N],
    is_core bool [N], num_clusters int32 [B]); cloud c's labels are its own
    (-1 noise, else 0..K_c-1) and equal what dbscan() gives for it alone.
    Asynchronous: nothing waits for the GPU.
    """
    import torch

    pts = points.contiguous()
    if pts.dtype != torch.float32 or pts.dim() != 2 or pts.shape[1] not in (2, 3):
        raise ValueError("points must be float32 with shape [N, 2] or [N, 3]")
    n, d = pts.shape
    dev = pts.device
    offs = offsets.to(device=dev, dtype=torch.int64).contiguous()
    b = offs.numel() - 1
    e = eps.to(device=dev, dtype=torch.float32).contiguous()
    mp = min_pts.to(device=dev, dtype=torch.int32).contiguous()
    if e.numel() != b or mp.numel() != b:
        raise ValueError("eps and min_pts need one entry per cloud")
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    h = handle if handle is not None else default_handle(idx)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    if is_core is None:
        is_core = torch.empty(n, dtype=torch.uint8, device=dev)
    _check_out(labels, is_core, n)
    if num_clusters is None:
        num_clusters = torch.empty(b, dtype=torch.int32, device=dev)
    opt = make_options(algo, border, leaf_size, block_size, tile=tile, graph=graph, validate=validate)
    stream = torch.cuda.current_stream(dev).cuda_stream
    ws_ptr, ws_size = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    h.dbscan_batched_raw(pts.data_ptr() if n else 0, n, offs.data_ptr(), b, d, e.data_ptr(), mp.data_ptr(),
                         labels.data_ptr() if n else 0, is_core.data_ptr() if n else 0, num_clusters.data_ptr(),
                         stream, opt, ws_ptr, ws_size)
    return labels, is_core.view(torch.bool), num_clusters


def dbscan_batched_host(points, offsets, eps, min_pts, budget_bytes: int, algo: str = "densebox",
                        border: str = "canonical", leaf_size: int = 0, block_size: int = 0, device: int = 0,
                        handle: Handle | None = None, labels=None, is_core=None, num_clusters=None):
    """Cluster a batch of clouds held in host memory, possibly more than fits on the
    device, within budget_bytes of device memory (groups of whole clouds, input
    copies overlapping the clustering of the previous group). Synchronous.

    points: [N, d] float32 host array (numpy or CPU torch tensor; pinned memory
    lets the copies overlap); offsets int64 [B+1]; eps float32 [B]; min_pts int32
    [B]. Returns (labels int32 [N], is_core uint8 [N], num_clusters int32 [B]) as
    numpy arrays (or the caller's own host buffers, filled), equal to what
    dbscan_batched gives for the same clouds.
    """
    import numpy as np

    def host(a, dtype):
        if hasattr(a, "numpy"):  # torch tensor
            if a.device.type != "cpu":
                raise TypeError("dbscan_batched_host takes host (CPU) arrays")
            a = a.numpy()
        a = np.asarray(a)
        if a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
            raise ValueError(f"expected a contiguous {np.dtype(dtype).name} array")
        return a

    pts = host(points, np.float32)
    if pts.ndim != 2 or pts.shape[1] not in (2, 3):
        raise ValueError("points must have shape [N, 2] or [N, 3]")
    offs, e, mp = host(offsets, np.int64), host(eps, np.float32), host(min_pts, np.int32)
    b = offs.shape[0] - 1
    if b < 1 or e.shape[0] != b or mp.shape[0] != b or offs[-1] != pts.shape[0]:
        raise ValueError("offsets must be [B+1] ending at N; eps and min_pts [B]")
    n = pts.shape[0]
    lab = np.empty(n, dtype=np.int32) if labels is None else host(labels, np.int32)
    core = np.empty(n, dtype=np.uint8) if is_core is None else host(is_core, np.uint8)
    k = np.empty(b, dtype=np.int32) if num_clusters is None else host(num_clusters, np.int32)
    if lab.shape[0] < n or core.shape[0] < n or k.shape[0] < b:
        raise ValueError("output buffers too small")
    h = handle if handle is not None else default_handle(device)
    opt = make_options(algo, border, leaf_size, block_size)
    h.dbscan_batched_host_raw(pts.ctypes.data if n else 0, offs.ctypes.data, b, pts.shape[1], e.ctypes.data,
                              mp.ctypes.data, int(budget_bytes), lab.ctypes.data if n else 0,
                              core.ctypes.data if n else 0, k.ctypes.data, opt)
    return lab, core, k


def tune(points, eps: float, min_pts: int, algo: str = "densebox", border: str = "canonical", reps: int = 3,
         handle: Handle | None = None, workspace=None):
    """fdb_tune on a torch tensor: times launch shapes on this input and keeps the
    fastest in the handle (and in the FDB_TUNE_CACHE file, if set) for later calls
    of the same class. Returns (options dict, best ms, default-shape ms)."""
    import torch

    pts = points.contiguous()
    n, d = pts.shape
    dev = pts.device.index if pts.device.index is not None else torch.cuda.current_device()
    h = handle if handle is not None else default_handle(dev)
    labels = torch.empty(n, dtype=torch.int32, device=pts.device)
    core = torch.empty(n, dtype=torch.uint8, device=pts.device)
    stream = torch.cuda.current_stream(pts.device).cuda_stream
    ws_ptr, ws_size = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    best, ms, ms0 = h.tune_raw(pts.data_ptr(), n, d, eps, min_pts, labels.data_ptr(), core.data_ptr(), stream,
                               make_options(algo, border), reps, ws_ptr, ws_size)
    return options_dict(best), ms, ms0


def tune_batched(points, offsets, eps, min_pts, algo: str = "densebox", border: str = "canonical", reps: int = 3,
                 handle: Handle | None = None, workspace=None):
    """fdb_tune_batched on torch tensors (as dbscan_batched). Returns (options dict,
    best ms, default-shape ms)."""
    import torch

    pts = points.contiguous()
    n, d = pts.shape
    dev = pts.device
    offs = offsets.to(device=dev, dtype=torch.int64).contiguous()
    b = offs.numel() - 1
    e = eps.to(device=dev, dtype=torch.float32).contiguous()
    mp = min_pts.to(device=dev, dtype=torch.int32).contiguous()
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    h = handle if handle is not None else default_handle(idx)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    ncl = torch.empty(b, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    ws_ptr, ws_size = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    best, ms, ms0 = h.tune_batched_raw(pts.data_ptr(), n, offs.data_ptr(), b, d, e.data_ptr(), mp.data_ptr(),
                                       labels.data_ptr(), core.data_ptr(), ncl.data_ptr(), stream,
                                       make_options(algo, border), reps, ws_ptr, ws_size)
    return options_dict(best), ms, ms0
