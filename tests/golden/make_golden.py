"""Write full-size expected values for the configured workloads.

Calls only the CPU oracle (and the seeded generators): for each workload it
stores the canonical labels' and core flags' SHA-256 (int32 / uint8, little
endian), K, the core / border / noise counts, and the neighbour-count sums
used by the cost model (sum |N_eps(x)| and sum min(|N_eps(x)|, minPts)).

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
from workloads.gen import CONFIGS, workload  # noqa: E402


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


def main(names):
    for name in names or list(CONFIGS):
        out = summarize(name)
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
