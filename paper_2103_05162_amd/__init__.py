"""Tree-based DBSCAN (FDbscan and FDbscan-DenseBox) for 2D/3D float32 points on
AMD Instinct MI355X, after Prokopenko, Lebrun-Grandie and Arndt, "Fast
tree-based algorithms for DBSCAN for low-dimensional data on GPUs" (ICPP 2023).

The clustering runs entirely in libfdbscan's HIP kernels (C ABI in
include/fdbscan.h); this package marshals torch tensors into that ABI.
"""
from __future__ import annotations

from ._lib import (FDB_INFO_DENSEBOX_FALLBACK, FDB_INFO_NONFINITE, FdbError, Handle, load, make_options,
                   status_string, workspace_bytes)

__all__ = ["dbscan", "Handle", "FdbError", "workspace_bytes", "default_handle", "load", "make_options",
           "status_string", "FDB_INFO_DENSEBOX_FALLBACK", "FDB_INFO_NONFINITE"]

_handles: dict[int, Handle] = {}


def default_handle(device: int = 0) -> Handle:
    h = _handles.get(device)
    if h is None:
        h = Handle(device)
        _handles[device] = h
    return h


def dbscan(points, eps: float, min_pts: int, algo: str = "fdbscan", border: str = "canonical",
           leaf_size: int = 0, block_size: int = 0, handle: Handle | None = None, labels=None, is_core=None,
           want_k: bool = True, workspace=None):
    """Cluster points ([n, 2] or [n, 3] float32 torch tensor on a HIP device).

    Returns (labels int32 [n], is_core bool [n], K). labels are in input order:
    -1 noise, else a cluster id 0..K-1 (canonical order unless border="first").
    K is None when want_k is False (then the call does not wait for the GPU).
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
    opt = make_options(algo, border, leaf_size, block_size)
    stream = torch.cuda.current_stream(pts.device).cuda_stream
    ws_ptr, ws_size = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    k = h.dbscan_raw(pts.data_ptr() if n else 0, n, d, eps, min_pts, labels.data_ptr() if n else 0,
                     is_core.data_ptr() if n else 0, stream, opt, want_k, ws_ptr, ws_size)
    return labels, is_core.bool(), k
