#!/usr/bin/env python3
"""Benchmark: DBSCAN throughput on one MI355X.

One step = one full clustering of the workload (every stage from device-resident
float32 points to device-resident int32 labels: bounds, keys, sort, gather,
LBVH, core pass, fused union traversal, finalisation, canonical ids, border pass,
scatter). The workload is the dense-clump 3D set: 8,388,608 points, 500 clumps
of sigma 5e-4 holding 80% of them, uniform background, eps = 0.002, minPts = 10.
DenseBox is the headline algorithm; FDbscan is measured beside it.

Prints one JSON line. `roofline` describes the dominant kernel (its duration is
measured with HIP events on the library's stream over the timed steps);
`cpu_baseline` times the CPU oracle on a spatial window of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 78.6          # fp32 vector lane-ops/s (256 CU x 4 SIMD x 16 lanes x 2 (dual-issue/packed) x 2.4 GHz)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", default="both", choices=["both", "densebox", "fdbscan"])
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1 = full 8M points)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=float, default=1 / 32,
                    help="volume fraction of the spatial window the CPU oracle clusters")
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    return ap.parse_args()


def time_algo(fdb, h, pts, eps, min_pts, algo, steps, warmup, leaf, block):
    import torch
    n = pts.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=pts.device)
    core = torch.empty(n, dtype=torch.uint8, device=pts.device)
    ws = torch.empty(fdb.workspace_bytes(n, 3, algo), dtype=torch.uint8, device=pts.device)
    kw = dict(algo=algo, handle=h, labels=labels, is_core=core, workspace=ws, leaf_size=leaf, block_size=block)
    _, _, k = fdb.dbscan(pts, eps, min_pts, **kw)          # also the K check
    for _ in range(warmup):
        fdb.dbscan(pts, eps, min_pts, want_k=False, **kw)
    torch.cuda.synchronize()
    h.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fdb.dbscan(pts, eps, min_pts, want_k=False, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, calls = h.stage_times()
    h.set_timing(False)
    ms = (t1 - t0) * 1e3 / steps
    per_call = {k2: v / max(calls, 1) for k2, v in stages.items()}
    return dict(ms=ms, k=k, stages=per_call, info=h.last_info())


def cpu_baseline(points, eps, min_pts, frac):
    import oracle
    from workloads.gen import window
    sample = window(points, frac)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    oracle.dbscan(sample, eps, min_pts, threads=cores)
    t = time.perf_counter() - t0
    return {"value": round(sample.shape[0] / t / 1e6, 4), "unit": "Mpts/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample.shape[0]} points in the corner window holding {frac:.4g} of the bounding volume "
                      f"(same local density), {t:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        log(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
            "the method here is single-device and no multi-GPU path is built.")
        sys.exit(2)
    import torch
    import paper_2103_05162_amd as fdb
    from workloads.gen import workload

    w = workload("c3_dense3d_8m", args.scale)
    log(f"[bench] workload {w.name}: n={w.n} eps={w.eps} minPts={w.min_pts}")
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(w.points).to(dev)
    h = fdb.Handle(0)
    algos = ["densebox", "fdbscan"] if args.algo == "both" else [args.algo]
    res = {}
    for a in algos:
        log(f"[bench] timing {a}: warmup {args.warmup}, steps {args.steps}")
        res[a] = time_algo(fdb, h, pts, w.eps, w.min_pts, a, args.steps, args.warmup, args.leaf_size,
                           args.block_size)
        r = res[a]
        log(f"[bench] {a}: {r['ms']:.3f} ms/step, K={r['k']}, info={r['info']}")
        for st, v in sorted(r["stages"].items(), key=lambda kv: -kv[1]):
            log(f"    {st:12s} {v:9.3f} ms")
    head = algos[0]
    ms = res[head]["ms"]
    out = {
        "metric": "Mpts/s clustered (3D, 8M pts)",
        "value": round(w.n / (ms / 1e3) / 1e6, 3),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} 3D float32 points, 500 Gaussian clumps (sigma 5e-4, 80%) "
                               f"+ uniform background, eps={w.eps:g}, minPts={w.min_pts}",
                   "algo": head, "num_clusters": res[head]["k"]},
        "stages_ms": {a: {k2: round(v, 4) for k2, v in res[a]["stages"].items()} for a in algos},
        "per_algo": {a: {"ms_per_step": round(res[a]["ms"], 4),
                         "mpts_per_s": round(w.n / (res[a]["ms"] / 1e3) / 1e6, 3),
                         "mfeatures_per_s": round(3 * w.n / (res[a]["ms"] / 1e3) / 1e6, 3),
                         "num_clusters": res[a]["k"]} for a in algos},
    }
    if not args.no_cpu_baseline:
        log(f"[bench] cpu oracle on a {args.cpu_window:g} window")
        out["cpu_baseline"] = cpu_baseline(w.points, w.eps, w.min_pts, args.cpu_window)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
