"""Comparison helpers shared by the oracle pins and the GPU parity tests.

None of these compute a clustering: they compare two label vectors, or pick
inputs for which an fp64 library result must agree with the fp32 test.
"""
from __future__ import annotations

import numpy as np


def partition_map(a: np.ndarray, b: np.ndarray, mask: np.ndarray) -> dict | None:
    """If labels a and b, restricted to mask, describe the same partition, return
    the bijection a-id -> b-id; otherwise None."""
    a = np.asarray(a)[mask]
    b = np.asarray(b)[mask]
    if a.size == 0:
        return {}
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    if len(np.unique(pairs[:, 0])) != len(pairs) or len(np.unique(pairs[:, 1])) != len(pairs):
        return None
    return {int(x): int(y) for x, y in pairs}


def same_partition(a, b, mask=None) -> bool:
    a = np.asarray(a)
    if mask is None:
        mask = np.ones(a.shape[0], dtype=bool)
    return partition_map(a, b, mask) is not None


def pick_safe_eps(points: np.ndarray, target: float, rel_gap: float = 1e-5) -> float:
    """An fp32 eps close to target such that no pairwise fp64 distance lies
    within rel_gap of it. Far from the threshold, the fp32 neighbour test and an
    fp64 library distance decide every pair the same way."""
    p = points.astype(np.float64)
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    d = np.sort(d[np.triu_indices(len(p), 1)])
    for k in range(1000):
        for sgn in (1, -1):
            e = float(np.float32(target * (1 + sgn * 3e-5 * k)))
            lo = np.searchsorted(d, e * (1 - rel_gap))
            hi = np.searchsorted(d, e * (1 + rel_gap))
            if lo == hi:
                return e
    raise RuntimeError("no safe eps found")


def assert_tolerance_mode(points, eps, labels, core, ref_labels, ref_core, check_border_fn):
    """Equality up to the free choice of a border point's cluster: core flags
    equal, noise equal, core partition equal up to renaming, and every border
    point sits in a cluster holding a core point within eps (checked by the
    given oracle checker)."""
    labels = np.asarray(labels)
    ref_labels = np.asarray(ref_labels)
    core = np.asarray(core, dtype=bool)
    ref_core = np.asarray(ref_core, dtype=bool)
    assert np.array_equal(core, ref_core), f"core flags differ at {np.flatnonzero(core != ref_core)[:10]}"
    assert np.array_equal(labels < 0, ref_labels < 0), "noise sets differ"
    assert same_partition(labels, ref_labels, core), "core partitions differ"
    assert check_border_fn(points, eps, core, labels) == 0, "a border point is in a cluster out of reach"
