"""Write full-size expected values for the configured workloads.

Calls only the CPU oracle (and the seeded generators): for each workload it
stores the canonical labels' and core flags' SHA-256 (int32 / uint8, little
endian), K, the core / border / noise counts, and the neighbour-count sums
used by the cost model (sum |N_eps(x)| and sum min(|N_eps(x)|, minPts)).

Two more files cover the many-cloud workloads, cloud by cloud:
  * c4_batched_4096: every cloud of the 4096-cloud batch, K and the first 16 hex
    digits of the SHA-256 of its canonical labels and core flags;
  * c5_served_sample: the same for a fixed sample of requests of the served trace
    (the requests' clouds, eps and minPts as the trace draws them), drawn among
    the requests of at most 65,536 points.

    python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads.gen import CONFIGS, batched_clouds, served_trace, workload  # noqa: E402

# the served trace as the benchmark replays it, and the requests sampled from it
SERVED = dict(requests=22000, rate=2000.0, pool_per_dim=128)
SERVED_WARM_S = 1.0
SERVED_SAMPLE = 48
SERVED_MAX_N = 65536


def summarize(name: str) -> dict:
    w = workload(name)
    threads = len(os.sched_getaffinity(0))
    t0 = time.time()
    labels, core, k = oracle.dbscan(w.points, w.eps, w.min_pts, method="grid", threads=threads)
    t1 = time.time()
    counts = oracle.neighbor_counts(w.points, w.eps, method="grid", threads=threads).astype(np.int64)
    t2 = time.time()
    return {
        "workload": name, "n": w.n, "dim": w.dim, "eps": w.eps, "min_pts": w.min_pts,
        "num_clusters": k, "num_core": int(core.sum()), "num_noise": int((labels < 0).sum()),
        "num_border": int(((~core) & (labels >= 0)).sum()),
        "labels_sha256": hashlib.sha256(labels.astype("<i4").tobytes()).hexdigest(),
        "core_sha256": hashlib.sha256(core.astype(np.uint8).tobytes()).hexdigest(),
        "points_sha256": hashlib.sha256(w.points.astype("<f4").tobytes()).hexdigest(),
        "sum_neighbors": int(counts.sum()),
        "sum_min_neighbors_minpts": int(np.minimum(counts, w.min_pts).sum()),
        "numpy": np.__version__,
        "oracle_seconds": round(t1 - t0, 2), "count_seconds": round(t2 - t1, 2), "threads": threads,
    }


def _sha16(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()[:16]


def _cloud_entry(pts, eps, mp, threads):
    labels, core, k = oracle.dbscan(pts, float(eps), int(mp), method="auto", threads=threads)
    return [int(k), _sha16(labels.astype("<i4")), _sha16(core.astype(np.uint8))]


def summarize_batched() -> dict:
    threads = len(os.sched_getaffinity(0))
    clouds, eps, mp = batched_clouds(4096)
    t0 = time.time()
    per = []
    for c, pts in enumerate(clouds):
        per.append(_cloud_entry(pts, eps[c], mp[c], threads))
        if c % 512 == 511:
            print(f"  c4: {c + 1} clouds, {time.time() - t0:.0f} s", flush=True)
    return {"workload": "c4_batched_4096", "num_clouds": len(clouds), "n": int(sum(len(c) for c in clouds)),
            "eps_sha256": hashlib.sha256(eps.astype("<f4").tobytes()).hexdigest(),
            "points_sha256_first_cloud": hashlib.sha256(clouds[0].astype("<f4").tobytes()).hexdigest(),
            "clouds": per, "oracle_seconds": round(time.time() - t0, 1), "threads": threads}


def served_sample_indices(arrival, n):
    """A fixed sample of the counted requests (after the warm-up) among those of at
    most SERVED_MAX_N points: the oracle's union loop visits every eps-pair, and the
    largest requests' clumps hold ~10^12 of them."""
    first = int(np.searchsorted(arrival, SERVED_WARM_S))
    idx = np.arange(first, len(arrival))
    idx = idx[n[first:] <= SERVED_MAX_N]
    rng = np.random.default_rng(0)
    return np.sort(rng.choice(idx, size=SERVED_SAMPLE, replace=False))


def summarize_served() -> dict:
    threads = len(os.sched_getaffinity(0))
    pool, req = served_trace(**SERVED)
    idx = served_sample_indices(req["arrival_s"], req["n"])
    t0 = time.time()
    per = []
    for r in idx:
        d, c = int(req["dim"][r]), int(req["cloud"][r])
        k, ls, cs = _cloud_entry(pool[d][c], req["eps"][r], req["min_pts"][r], threads)
        per.append([int(r), d, c, int(req["n"][r]), k, ls, cs])
    return {"workload": "c5_served_sample", "trace": SERVED, "warm_s": SERVED_WARM_S, "max_n": SERVED_MAX_N,
            "requests": per, "oracle_seconds": round(time.time() - t0, 1), "threads": threads}


EXTRA = {"c4_batched_4096": summarize_batched, "c5_served_sample": summarize_served}


def main(names):
    for name in names or list(CONFIGS) + list(EXTRA):
        out = EXTRA[name]() if name in EXTRA else summarize(name)
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
