"""Seeded synthetic point-cloud generators.

These stand in for the paper's datasets (Table 1: GPS traces, HACC cosmology
particles, and generator-made similar/variable-density clusters), which are not
available here. Each generator draws Gaussian clumps of varying density over a
uniform background in 2D or 3D, the structure those datasets share.

This module holds no DBSCAN arithmetic: it only produces inputs (points, eps,
minPts). Both the CPU oracle and the GPU path consume its output.

Rules common to every generator:
  * numpy.random.default_rng(seed) (PCG64); coordinates drawn in float64 and
    cast to float32 at the end;
  * clump centres uniform in the domain, no clamping (Gaussian tails may leave
    the domain);
  * the final point order is shuffled with the same generator.

`scale` (0 < scale <= 1) shrinks a workload while keeping its local density:
the point count and the number of clumps are multiplied by `scale`, and the
domain side by scale**(1/d), so clump sizes, background density and eps stay
the same. scale=1 is the full workload.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    points: np.ndarray  # [n, d] float32, row-major
    eps: float
    min_pts: int

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def dim(self) -> int:
        return int(self.points.shape[1])


def _finish(rng: np.random.Generator, parts: list[np.ndarray], d: int) -> np.ndarray:
    pts = np.concatenate(parts, axis=0) if parts else np.zeros((0, d))
    pts = pts[rng.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts.astype(np.float32))


def blobs_2d(seed: int = 1, n: int = 16384, n_blobs: int = 8, sigma: float = 0.01,
             clump_frac: float = 0.7, scale: float = 1.0) -> np.ndarray:
    """2D: floor(clump_frac*n) points split equally over isotropic Gaussian blobs
    (remainder to the last blob), the rest uniform in the square."""
    d = 2
    rng = np.random.default_rng(seed)
    n = max(0, int(round(n * scale)))
    n_blobs = max(1, int(round(n_blobs * scale)))
    side = scale ** (1.0 / d)
    n_clump = int(math.floor(clump_frac * n))
    centers = rng.uniform(0.0, side, size=(n_blobs, d))
    sizes = np.full(n_blobs, n_clump // n_blobs)
    sizes[-1] += n_clump - sizes.sum()
    parts = [centers[b] + sigma * rng.standard_normal((int(sizes[b]), d)) for b in range(n_blobs)]
    parts.append(rng.uniform(0.0, side, size=(n - n_clump, d)))
    return _finish(rng, parts, d)


def lognormal_clumps_3d(seed: int = 2, n: int = 2_097_152, n_clumps: int = 2000,
                        bg_frac: float = 0.2, sigma_lo: float = 0.002, sigma_hi: float = 0.02,
                        scale: float = 1.0) -> np.ndarray:
    """3D friends-of-friends style: a uniform background fraction plus clumps whose
    member counts follow LogNormal(0,1) weights (multinomial split) and whose
    widths are log-normal with median sqrt(sigma_lo*sigma_hi), log-sd chosen so
    that the clip range [sigma_lo, sigma_hi] is +-2 log-sd."""
    d = 3
    rng = np.random.default_rng(seed)
    n = max(0, int(round(n * scale)))
    n_clumps = max(1, int(round(n_clumps * scale)))
    side = scale ** (1.0 / d)
    n_bg = int(round(bg_frac * n))
    n_clump = n - n_bg
    w = rng.lognormal(0.0, 1.0, size=n_clumps)
    sizes = rng.multinomial(n_clump, w / w.sum())
    med = math.sqrt(sigma_lo * sigma_hi)
    logsd = math.log(sigma_hi / med) / 2.0
    sig = np.clip(rng.lognormal(math.log(med), logsd, size=n_clumps), sigma_lo, sigma_hi)
    centers = rng.uniform(0.0, side, size=(n_clumps, d))
    parts = [centers[c] + sig[c] * rng.standard_normal((int(sizes[c]), d)) for c in range(n_clumps)]
    parts.append(rng.uniform(0.0, side, size=(n_bg, d)))
    return _finish(rng, parts, d)


def dense_clumps_3d(seed: int = 3, n: int = 8_388_608, n_clumps: int = 500, sigma: float = 5e-4,
                    clump_frac: float = 0.8, scale: float = 1.0) -> np.ndarray:
    """3D dense-box stress: floor(clump_frac*n) points in equal very dense clumps
    (remainder to the last), the rest uniform in the cube."""
    d = 3
    rng = np.random.default_rng(seed)
    n = max(0, int(round(n * scale)))
    n_clumps = max(1, int(round(n_clumps * scale)))
    side = scale ** (1.0 / d)
    n_clump = int(math.floor(clump_frac * n))
    centers = rng.uniform(0.0, side, size=(n_clumps, d))
    sizes = np.full(n_clumps, n_clump // n_clumps)
    sizes[-1] += n_clump - sizes.sum()
    parts = [centers[c] + sigma * rng.standard_normal((int(sizes[c]), d)) for c in range(n_clumps)]
    parts.append(rng.uniform(0.0, side, size=(n - n_clump, d)))
    return _finish(rng, parts, d)


def mixture_cloud(rng: np.random.Generator, n: int, d: int = 3, k_max: int = 20,
                  sigma_lo: float = 0.002, sigma_hi: float = 0.02, noise_frac: float = 0.1) -> np.ndarray:
    """One cloud of a batch: k ~ U{1..k_max} Gaussian clumps with log-uniform widths
    holding (1-noise_frac) of the points (equal split, remainder to the last), the
    rest uniform in the unit cube."""
    k = int(rng.integers(1, k_max + 1))
    n_noise = int(round(noise_frac * n))
    n_clump = n - n_noise
    sig = np.exp(rng.uniform(math.log(sigma_lo), math.log(sigma_hi), size=k))
    centers = rng.uniform(0.0, 1.0, size=(k, d))
    sizes = np.full(k, n_clump // k)
    sizes[-1] += n_clump - sizes.sum()
    parts = [centers[c] + sig[c] * rng.standard_normal((int(sizes[c]), d)) for c in range(k)]
    parts.append(rng.uniform(0.0, 1.0, size=(n_noise, d)))
    return _finish(rng, parts, d)


def batched_clouds(num_clouds: int = 4096, seed: int = 4, lo: int = 1024, hi: int = 65536,
                   eps_lo: float = 0.005, eps_hi: float = 0.02, min_pts: int = 5):
    """Many independent 3D clouds; cloud c draws from SeedSequence([seed, c]).
    Returns (list of [n_c,3] float32 arrays, eps per cloud (float32), minPts per cloud)."""
    clouds, eps, mp = [], [], []
    for c in range(num_clouds):
        rng = np.random.default_rng(np.random.SeedSequence([seed, c]))
        n_c = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        e = float(np.float32(rng.uniform(eps_lo, eps_hi)))
        clouds.append(mixture_cloud(rng, n_c))
        eps.append(e)
        mp.append(min_pts)
    return clouds, np.asarray(eps, dtype=np.float32), np.asarray(mp, dtype=np.int32)


def served_trace(seed: int = 5, requests: int = 22000, rate: float = 2000.0, pool_per_dim: int = 48,
                 lo: int = 10240, hi: int = 2097152, eps_lo: float = 0.005, eps_hi: float = 0.02,
                 min_pts=(2, 5, 10)):
    """Open-loop request stream for a clustering server: Poisson arrivals at `rate`
    per second; each request draws d in {2, 3}, minPts from `min_pts` and eps
    ~ U[eps_lo, eps_hi], and names one cloud of a resident pool (pool_per_dim
    clouds per dimension, sizes floor(exp U(ln lo, ln hi)), drawn with
    mixture_cloud), so request sizes follow the same log-uniform law.
    Returns (pool: {2: [arrays], 3: [arrays]}, requests: dict of numpy arrays
    arrival_s, dim, cloud, eps, min_pts, n)."""
    rng = np.random.default_rng(seed)
    pool = {}
    for d in (2, 3):
        pool[d] = []
        for c in range(pool_per_dim):
            crng = np.random.default_rng(np.random.SeedSequence([seed, d, c]))
            n_c = int(math.floor(math.exp(crng.uniform(math.log(lo), math.log(hi)))))
            pool[d].append(mixture_cloud(crng, n_c, d=d))
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=requests))
    dim = rng.choice([2, 3], size=requests).astype(np.int32)
    cloud = rng.integers(0, pool_per_dim, size=requests).astype(np.int32)
    eps = rng.uniform(eps_lo, eps_hi, size=requests).astype(np.float32)
    mp = rng.choice(np.asarray(min_pts, dtype=np.int32), size=requests).astype(np.int32)
    n = np.array([pool[int(d)][int(c)].shape[0] for d, c in zip(dim, cloud)], dtype=np.int64)
    return pool, {"arrival_s": arrival, "dim": dim, "cloud": cloud, "eps": eps, "min_pts": mp, "n": n}


# The three single-cloud workloads (name -> (generator, eps, minPts)).
CONFIGS = {
    "c1_blobs2d_16k": (blobs_2d, 0.01, 5),
    "c2_fof3d_2m": (lognormal_clumps_3d, 0.005, 2),
    "c3_dense3d_8m": (dense_clumps_3d, 0.002, 10),
}


def workload(name: str, scale: float = 1.0) -> Workload:
    gen, eps, mp = CONFIGS[name]
    pts = gen(scale=scale)
    tag = name if scale == 1.0 else f"{name}@{scale:g}"
    return Workload(tag, pts, float(np.float32(eps)), mp)


def window(points: np.ndarray, frac: float) -> np.ndarray:
    """Points inside the corner sub-box [0, frac**(1/d) * extent] of the bounding
    box: a spatial sample with the workload's local density."""
    d = points.shape[1]
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    cut = lo + (hi - lo) * frac ** (1.0 / d)
    keep = np.all(points <= cut, axis=1)
    return np.ascontiguousarray(points[keep])
