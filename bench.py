#!/usr/bin/env python3
"""Benchmark: DBSCAN throughput on one MI355X.

One step = one full clustering of the workload (every stage from device-resident
float32 points to device-resident int32 labels: bounds, keys, sort, gather,
LBVH, core pass, fused union traversal, finalisation, canonical ids, border pass,
scatter). The headline workload is the dense-clump 3D set: 8,388,608 points, 500
clumps of sigma 5e-4 holding 80% of them, uniform background, eps = 0.002,
minPts = 10. DenseBox is the headline algorithm; FDbscan is measured beside it,
and both run on the 2,097,152-point friends-of-friends set (eps 0.005, minPts 2)
and the 16,384-point 2D blob set (eps 0.01, minPts 5). Each single-cloud leg
checks its labels against the oracle's stored hashes and reports the dominant
kernel's roofline fraction and the whole pipeline's (compulsory bytes over the
step time against 8 TB/s); with --tune it also runs the autotuner and times the
tuned launch shape.

A batched leg clusters 4096 uneven 3D clouds (1024-65535 points each, every
cloud with its own eps) in one call, replays the same call from a recorded HIP
graph, and reports clouds/s beside a loop of one call per cloud over the same
data, whether all give identical labels, and how many clouds match the oracle's
stored per-cloud hashes.

A served leg replays an open-loop request stream (Poisson arrivals, clouds of
10k-2M points, 2D and 3D, mixed eps and minPts) against the continuous-batching
server at two offered rates and against a plain one-job-at-a-time server, and
reports p50/p99 latency, throughput and whether each keeps up.

Prints one JSON line. `cpu_baseline` times the CPU oracle on a spatial window of
the headline set; `cpu_oracle_full` times it on the two smaller sets whole, at
every usable core and at one thread, with the CPU model.
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
# fp32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s for the plain
# (non-packed, non-fused) v_sub/v_mul/v_add/v_cmp the neighbour test compiles to; packed
# fp32 would double it (78.6 T) but is disabled in this build. The published 157.3 TFLOP/s
# counts a packed FMA as 4 flops.
ALU_PEAK_TOPS = 39.3
ALU_PEAK_PACKED_TOPS = 78.6


def pred_ops(d):
    """fp32 operations of one neighbour test: d subtractions, d products, d-1 sums, one compare."""
    return 3 * d


def unit_sizes(d):
    """Bytes per unit at the reference layout: point P, Morton code C, index I, internal
    node N (box + two child links), flag F."""
    return dict(P=4 * d, C=8, I=4, N=8 * d + 8, F=1)


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
    ap.add_argument("--cpu-window", type=float, default=1 / 8,
                    help="volume fraction of the spatial window the CPU oracle clusters")
    ap.add_argument("--batched-algo", default="densebox", choices=["none", "densebox", "fdbscan"],
                    help="algorithm of the batched many-cloud leg (none = skip it)")
    ap.add_argument("--clouds", type=int, default=4096, help="clouds in the batched leg")
    ap.add_argument("--loop-passes", type=int, default=1,
                    help="timed passes of the one-call-per-cloud loop beside the batch (0 = skip it)")
    ap.add_argument("--served-algo", default="densebox", choices=["none", "densebox", "fdbscan"],
                    help="algorithm of the served leg (none = skip it)")
    ap.add_argument("--requests", type=int, default=22000, help="requests in the served trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="request arrivals per second")
    ap.add_argument("--extra-rates", type=float, nargs="*", default=[4000.0],
                    help="further offered rates for the continuous-batching server")
    ap.add_argument("--no-small-legs", action="store_true", help="skip the 2M-point and 16k-point workloads")
    ap.add_argument("--tune", action=argparse.BooleanOptionalAction, default=True,
                    help="also run the autotuner and time the tuned launch shape")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="HBM budget of the served batches")
    ap.add_argument("--pool-per-dim", type=int, default=128, help="resident clouds per dimension")
    ap.add_argument("--ooc-budget-gib", type=float, default=6.0,
                    help="device budget of the out-of-core batched leg (0 = skip it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run kernels of known traffic on this many MiB (PMC calibration): a "
                         "device-to-device copy, and gathers of 12-byte rows by identity and random index")
    return ap.parse_args()


def time_algo(fdb, h, pts, eps, min_pts, algo, steps, warmup, leaf=0, block=0):
    """Time `steps` calls of one algorithm on device-resident points (HIP-event stage
    timing off), then the same number with stage timing on for the per-stage
    breakdown. Returns ms per step, K, stage ms per call, info bits and sizes."""
    import torch
    n, d = pts.shape
    labels = torch.empty(n, dtype=torch.int32, device=pts.device)
    core = torch.empty(n, dtype=torch.uint8, device=pts.device)
    ws = torch.empty(fdb.workspace_bytes(n, d, algo), dtype=torch.uint8, device=pts.device)
    kw = dict(algo=algo, handle=h, labels=labels, is_core=core, workspace=ws, leaf_size=leaf, block_size=block)
    _, _, k = fdb.dbscan(pts, eps, min_pts, **kw)          # also the K check
    for _ in range(warmup):
        fdb.dbscan(pts, eps, min_pts, want_k=False, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fdb.dbscan(pts, eps, min_pts, want_k=False, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    h.set_timing(True)
    for _ in range(steps):
        fdb.dbscan(pts, eps, min_pts, want_k=False, **kw)
    torch.cuda.synchronize()
    stages, calls = h.stage_times()
    h.set_timing(False)
    per_call = {k2: v / max(calls, 1) for k2, v in stages.items()}
    return dict(ms=ms, k=k, stages=per_call, info=h.last_info(), sizes=h.last_counts(),
                labels=labels, core=core)


def run_leg(fdb, h, name, algos, steps, warmup, scale=1.0, tune=False):
    """One single-cloud workload: every algorithm timed, its stages, its roofline."""
    import torch
    from workloads.gen import workload
    w = workload(name, scale)
    d = w.points.shape[1]
    pts = torch.from_numpy(w.points).to("cuda:0")
    golden = load_golden(name) if scale == 1.0 else None
    traffic_db = load_traffic() if name == "c3_dense3d_8m" and scale == 1.0 else None
    out = {"workload": w.name, "n": w.n, "dim": d, "eps": w.eps, "min_pts": w.min_pts, "algos": {}}
    for a in algos:
        log(f"[bench] {w.name} {a}: warmup {warmup}, steps {steps}")
        r = time_algo(fdb, h, pts, w.eps, w.min_pts, a, steps, warmup)
        rl, pipe = roofline(a, d, w.n, w.min_pts, r["stages"], r["ms"], r["sizes"], golden, traffic_db)
        ok = None
        if golden is not None:
            ok = (r["k"] == golden["num_clusters"] and
                  sha256(r["labels"].cpu().numpy()) == golden["labels_sha256"] and
                  sha256(r["core"].cpu().numpy().astype(np.uint8)) == golden["core_sha256"])
        log(f"[bench]   {r['ms']:.3f} ms/step, K={r['k']}, info={r['info']}, oracle labels matched: {ok}")
        for st, v in sorted(r["stages"].items(), key=lambda kv: -kv[1]):
            log(f"    {st:12s} {v:9.3f} ms")
        entry = {"ms_per_step": round(r["ms"], 4), "mpts_per_s": round(w.n / (r["ms"] / 1e3) / 1e6, 3),
                 "mfeatures_per_s": round(d * w.n / (r["ms"] / 1e3) / 1e6, 3), "num_clusters": r["k"],
                 "labels_match_oracle_golden": ok, "sizes": r["sizes"], "info": r["info"],
                 "stages_ms": {k2: round(v, 4) for k2, v in r["stages"].items()},
                 "roofline": rl, "pipeline": pipe}
        if tune:
            best, tms, dms = fdb.tune(pts, w.eps, w.min_pts, algo=a, reps=3, handle=h)
            r2 = time_algo(fdb, h, pts, w.eps, w.min_pts, a, steps, warmup)  # the handle now holds the shape
            entry["tuned"] = {"shape": {k2: best[k2] for k2 in ("leaf_size", "block_size", "tile")},
                              "ms_per_step": round(r2["ms"], 4), "default_ms_per_step": round(r["ms"], 4),
                              "tuner_best_ms": round(tms, 4), "tuner_default_ms": round(dms, 4),
                              "labels_equal_default": bool(torch.equal(r2["labels"], r["labels"]))}
            log(f"[bench]   tuned {entry['tuned']['shape']}: {r2['ms']:.3f} ms/step (default {r['ms']:.3f})")
        out["algos"][a] = entry
        del r
    return out


def sha256(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def time_batched(fdb, h, algo, steps, warmup, num_clouds, loop_passes, ooc_budget=0, tune=False):
    """Batched clustering of many uneven 3D clouds (each with its own eps and minPts)
    in one call, against the same clouds clustered one call at a time."""
    import torch
    from workloads.gen import batched_clouds
    t0 = time.perf_counter()
    clouds, eps, mp = batched_clouds(num_clouds)
    sizes = np.array([c.shape[0] for c in clouds], dtype=np.int64)
    offs = np.zeros(num_clouds + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    n = int(offs[-1])
    log(f"[bench] batched workload: {num_clouds} clouds, {n} points ({time.perf_counter() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(np.concatenate(clouds)).to(dev)
    del clouds
    d_off = torch.from_numpy(offs).to(dev)
    d_eps = torch.from_numpy(eps).to(dev)
    d_mp = torch.from_numpy(mp).to(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    ncl = torch.empty(num_clouds, dtype=torch.int32, device=dev)
    ws = torch.empty(fdb.workspace_bytes_batched(n, num_clouds, 3, algo), dtype=torch.uint8, device=dev)
    kw = dict(algo=algo, handle=h, labels=labels, is_core=core, num_clusters=ncl, workspace=ws)
    for _ in range(max(warmup, 1)):
        fdb.dbscan_batched(pts, d_off, d_eps, d_mp, **kw)
    torch.cuda.synchronize()
    info = h.last_info()
    h.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fdb.dbscan_batched(pts, d_off, d_eps, d_mp, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stages, calls = h.stage_times()
    h.set_timing(False)
    # the same batch replayed from the handle's recorded HIP graph (one launch per call)
    ref_labels = labels.clone()
    fdb.dbscan_batched(pts, d_off, d_eps, d_mp, graph=True, **kw)   # records the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fdb.dbscan_batched(pts, d_off, d_eps, d_mp, graph=True, **kw)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / steps
    graph_same = bool(torch.equal(labels, ref_labels))
    tuned = None
    if tune:
        best, tms, dms = fdb.tune_batched(pts, d_off, d_eps, d_mp, algo=algo, reps=3, handle=h, workspace=ws)
        fdb.dbscan_batched(pts, d_off, d_eps, d_mp, **kw)  # the handle now holds the tuned shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fdb.dbscan_batched(pts, d_off, d_eps, d_mp, **kw)
        torch.cuda.synchronize()
        tuned = {"shape": {k2: best[k2] for k2 in ("leaf_size", "block_size", "tile")},
                 "ms_per_batch": round((time.perf_counter() - t0) * 1e3 / steps, 3), "default_ms_per_batch": round(ms, 3),
                 "tuner_best_ms": round(tms, 3), "tuner_default_ms": round(dms, 3),
                 "labels_equal_default": bool(torch.equal(labels, ref_labels))}
        log(f"[bench] batched tuned {tuned['shape']}: {tuned['ms_per_batch']} ms (default {ms:.3f})")
    ooc = None
    if ooc_budget > 0:
        # the same batch held in pinned host memory, clustered inside a device budget
        # smaller than the batch needs (copies over PCIe included)
        pts_h = pts.cpu().pin_memory()
        lab_h = torch.empty(n, dtype=torch.int32).pin_memory()
        core_h = torch.empty(n, dtype=torch.uint8).pin_memory()
        k_h = np.empty(num_clouds, np.int32)
        okw = dict(algo=algo, handle=h, labels=lab_h, is_core=core_h, num_clusters=k_h)
        fdb.dbscan_batched_host(pts_h, offs, eps, mp, ooc_budget, **okw)
        t0 = time.perf_counter()
        for _ in range(steps):
            fdb.dbscan_batched_host(pts_h, offs, eps, mp, ooc_budget, **okw)
        ooc_ms = (time.perf_counter() - t0) * 1e3 / steps
        same = bool(torch.equal(lab_h, labels.cpu()) and torch.equal(core_h, core.cpu()) and
                    np.array_equal(k_h, ncl.cpu().numpy()))
        ooc = dict(ms=ooc_ms, budget=ooc_budget, identical=same,
                   need=fdb.workspace_bytes_batched(n, num_clouds, 3, algo) + n * 17 + num_clouds * 20)
        del pts_h, lab_h, core_h
    # one call per cloud, outputs written in place, one workspace sized for the largest cloud
    opt = fdb.make_options(algo)
    lws = torch.empty(fdb.workspace_bytes(int(sizes.max()), 3, algo), dtype=torch.uint8, device=dev)
    lab2 = torch.empty_like(labels)
    core2 = torch.empty_like(core)
    stream = torch.cuda.current_stream(dev).cuda_stream
    bp, lp, cp, wp, wsz = pts.data_ptr(), lab2.data_ptr(), core2.data_ptr(), lws.data_ptr(), lws.numel()

    def loop():
        for c in range(num_clouds):
            b, nc = int(offs[c]), int(sizes[c])
            h.dbscan_raw(bp + 12 * b, nc, 3, float(eps[c]), int(mp[c]), lp + 4 * b, cp + b, stream, opt, False,
                         wp, wsz)

    common = dict(ms=ms, graph_ms=graph_ms, graph_identical=graph_same, tuned=tuned, n=n, info=info, ooc=ooc,
                  stages={k2: v / max(calls, 1) for k2, v in stages.items()}, clusters=int(ncl.sum().item()),
                  golden=golden_batch_check(labels, core, ncl, offs, sizes))
    if loop_passes <= 0:
        return dict(loop_ms=None, identical=None, **common)
    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_passes):
        loop()
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3 / loop_passes
    same = bool(torch.equal(labels, lab2) and torch.equal(core, core2))
    return dict(loop_ms=loop_ms, identical=same, **common)


def golden_batch_check(labels, core, ncl, offs, sizes):
    """Clouds whose K, labels and core flags match the oracle's stored per-cloud hashes
    (tests/golden/c4_batched_4096.json), when the batch is that workload."""
    g = load_golden("c4_batched_4096")
    if g is None or g["num_clouds"] != len(sizes) or g["n"] != int(offs[-1]):
        return None
    lab, co, kk = labels.cpu().numpy(), core.cpu().numpy().astype(np.uint8), ncl.cpu().numpy()
    good = 0
    for c, (k, ls, cs) in enumerate(g["clouds"]):
        sl = slice(int(offs[c]), int(offs[c + 1]))
        if (int(kk[c]) == k and sha256(lab[sl].astype("<i4"))[:16] == ls and sha256(co[sl])[:16] == cs):
            good += 1
    return {"clouds_matching_oracle": good, "clouds": len(g["clouds"])}


def replay(fdb, mode, algo, budget, max_batch, ptrs, req, out, warm_s):
    """Replay the request trace open-loop against one server; returns its stats over
    the requests that arrive after the warm-up period."""
    srv = fdb.Server(0, budget_bytes=budget, max_batch=max_batch, mode=mode, algo=algo)
    arrival, dim, n, eps, mp, off = (req["arrival_s"], req["dim"], req["n"], req["eps"], req["min_pts"],
                                     req["out_off"])
    first = int(np.searchsorted(arrival, warm_s))
    base = out.data_ptr()
    lag = 0.0
    t0 = time.perf_counter() + 0.05
    next_log = 2.0
    try:
        for r in range(len(arrival)):
            ta = t0 + arrival[r]
            now = time.perf_counter()
            while now < ta:
                now = time.perf_counter()
            lag = max(lag, now - ta)
            srv.submit_raw(ptrs[r], int(n[r]), int(dim[r]), float(eps[r]), int(mp[r]), base + 4 * int(off[r]))
            if arrival[r] >= next_log:
                log(f"[bench]   {mode}: {r + 1} requests submitted")
                next_log += 2.0
        srv.drain()
        st = srv.stats(first)
        st_all = srv.stats(0)
    finally:
        srv.close()
    window = float(arrival[-1] - arrival[first]) if len(arrival) > first + 1 else 0.0
    offered = (len(arrival) - first) / window if window > 0 else 0.0
    served = st["jobs"] / st["span_s"] if st["span_s"] > 0 else 0.0
    return {"p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
            "mean_ms": round(st["mean_us"] / 1e3, 3), "max_ms": round(st["max_us"] / 1e3, 3),
            "jobs_per_s": round(served, 1), "offered_jobs_per_s": round(offered, 1),
            "mpts_per_s": round(st["points"] / st["span_s"] / 1e6, 1) if st["span_s"] > 0 else 0.0,
            "saturated": bool(served < 0.95 * offered), "jobs": st["jobs"], "batches": st["batches"],
            "max_batch_jobs": st["max_batch_jobs"], "max_queue": st["max_queue"],
            "busy_frac": round(st_all["busy_s"] / st_all["span_s"], 3) if st_all["span_s"] > 0 else None,
            "client_lag_max_us": round(float(lag) * 1e6, 1)}


def time_served(fdb, algo, requests, rates, budget_gib, pool_per_dim, warm_s=1.0):
    """Served leg: the open-loop trace replayed on the continuous-batching server at
    each offered rate, and on the plain one-job-at-a-time server at the first rate;
    sampled requests' labels are compared between the two and with the oracle's
    stored hashes (tests/golden/c5_served_sample.json)."""
    import torch
    from workloads.gen import served_trace
    t0 = time.perf_counter()
    pool, req = served_trace(requests=requests, rate=rates[0], pool_per_dim=pool_per_dim)
    log(f"[bench] served trace: {requests} requests at {rates[0]:g}/s, pool of {2 * pool_per_dim} clouds "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    pool_dev = {d: [torch.from_numpy(c).to(dev) for c in pool[d]] for d in pool}
    del pool
    ptrs = [pool_dev[int(d)][int(c)].data_ptr() for d, c in zip(req["dim"], req["cloud"])]
    req["out_off"] = np.concatenate([[0], np.cumsum(req["n"])[:-1]]).astype(np.int64)
    total = int(req["n"].sum())
    out = torch.empty(total, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    budget = int(budget_gib * (1 << 30))
    base_arrival = req["arrival_s"].copy()
    first = int(np.searchsorted(base_arrival, warm_s))
    rng = np.random.default_rng(0)
    sample = rng.choice(np.arange(first, requests), size=min(64, requests - first), replace=False)
    g = load_golden("c5_served_sample")
    gmatch = g is not None and g["trace"] == {"requests": requests, "rate": rates[0], "pool_per_dim": pool_per_dim}
    gold_idx = [int(e[0]) for e in g["requests"]] if gmatch else []

    def grab(idx):
        return {int(r): out[int(req["out_off"][r]):int(req["out_off"][r]) + int(req["n"][r])].cpu() for r in idx}

    res, kept, golden_ok = {}, {}, None
    runs = [("batched", r) for r in rates] + [("fifo", rates[0])]
    for mode, rate in runs:
        req["arrival_s"] = base_arrival * (rates[0] / rate)   # the same draws at another offered rate
        key = f"{mode}@{rate:g}"
        log(f"[bench] serving the trace ({key})")
        out.fill_(-9)
        res[key] = replay(fdb, mode, algo, budget, 4096, ptrs, req, out, warm_s * rates[0] / rate)
        log(f"[bench]   {key}: {res[key]}")
        if rate == rates[0]:
            kept[mode] = grab(sample)
            if mode == "batched" and gmatch:
                got = grab(gold_idx)
                golden_ok = sum(sha256(got[int(e[0])].numpy().astype("<i4"))[:16] == e[5] for e in g["requests"])
    same = all(torch.equal(kept["batched"][r], kept["fifo"][r]) for r in kept["batched"])
    del out, pool_dev
    torch.cuda.empty_cache()
    b0 = res[f"batched@{rates[0]:g}"]
    f0 = res[f"fifo@{rates[0]:g}"]
    return {"workload": f"{requests} requests, Poisson arrivals (first {warm_s:g} s at {rates[0]:g}/s not counted), "
                        f"sizes log-uniform 10240-2097151 from a resident pool of {2 * pool_per_dim} clouds, "
                        f"d in {{2,3}}, minPts in {{2,5,10}}, eps 0.005-0.02",
            "algo": algo, "hbm_budget_gib": budget_gib, "mean_points": round(float(req["n"].mean()), 1),
            "rates": {k: v for k, v in res.items()},
            "batched": b0, "fifo": f0,
            "p99_speedup_vs_fifo": round(f0["p99_ms"] / b0["p99_ms"], 3) if b0["p99_ms"] > 0 else None,
            "identical_labels_sampled": same, "sampled_requests": len(sample),
            "oracle_golden_requests_matching": golden_ok,
            "oracle_golden_requests": len(gold_idx) if gmatch else None}


# The library's stage names that are one kernel launch each (the kernel rocprofv3 names).
SINGLE_KERNEL = {
    "densebox": {"core": "k_core_dbx", "main_cells": "k_main_dbx_cells_wave", "main_points": "k_main_dbx_points",
                 "permute": "k_permute", "finalize": "k_finalize"},
    "fdbscan": {"core": "k_core_fdb", "main": "k_main_fdb_q", "finalize": "k_finalize"},
}


def stage_bytes(algo, d, n, sizes, min_pts):
    """Compulsory HBM bytes of each step of the method for one call: every input read
    once and every output written once at the reference layout (the sort counts one
    read and one write of key and index, whatever its pass count; a traversal counts
    one read of the tree and points; cache reuse is free). Keyed by the library's
    stage names; the last entry covers the method's sort of the mixed primitives
    (DenseBox), which the one cell-key sort already yields here."""
    u = unit_sizes(d)
    P, C, I, N, F = u["P"], u["C"], u["I"], u["N"], u["F"]
    walk = P + F + N + P + F + I + 2 * I        # fused pass per query: point, flag, tree, neighbour, union
    core = P + N + P + F                        # early-exit count per query
    out = {"bounds": n * P, "permute": n * (I + 2 * P), "finalize": n * 2 * I,
           "cluster_ids": n * 2 * I, "scatter": n * 2 * I}
    if algo == "fdbscan":
        out.update({"morton": n * (P + C + I), "sort": 2 * n * (C + I), "lbvh": n * (C + P + N),
                    "main": n * walk})
        if min_pts > 2:
            out["core"] = n * core
        return out
    m, c = sizes["prims"], sizes["dense_cells"]
    ns = m - c                                  # points outside dense cells
    nd = n - ns                                 # points inside them
    out.update({"cell_keys": n * (P + 8 + I), "sort": 2 * n * (8 + I),
                "dense_cells": 8 * n + m * (P + C + I),   # run lengths, then the primitives' keys
                "lbvh": m * (C + P + N),
                "main_cells": nd * walk + 8 * nd,          # dense-cell points, plus the union inside each cell
                "main_points": ns * walk,
                "sort_of_primitives": 2 * m * (C + I)})
    if min_pts > 2:
        out["core"] = ns * core                           # the isolated-point test and the walks
    return out


def roofline(algo, d, n, min_pts, stages, step_ms, sizes, golden, traffic_db):
    """The dominant single-kernel stage against its roofline (its algorithmic bytes,
    or pair tests for the ALU-bound FDbscan walks, over its HIP-event duration), and
    the whole pipeline's algorithmic bytes over the step time."""
    sb = stage_bytes(algo, d, n, sizes, min_pts)
    total = sum(sb.values())
    t_roof_ms = total / (HBM_PEAK_GBS * 1e9) * 1e3
    pipeline = {"alg_bytes": int(total), "ms": round(step_ms, 4),
                "achieved": round(total / (step_ms / 1e3) / 1e9, 1), "unit": "GB/s",
                "frac": round(t_roof_ms / step_ms, 4), "t_roof_ms": round(t_roof_ms, 4)}
    single = SINGLE_KERNEL[algo]
    cand = {k: v for k, v in stages.items() if k in single}
    if not cand:
        return None, pipeline
    dom = max(cand, key=cand.get)
    ms = cand[dom]
    alu = (algo == "fdbscan" and dom in ("main", "core") and golden is not None
           and "sum_neighbors" in golden)
    if alu:
        # one neighbour test per pair in the masked main phase, up to minPts per point in the core pass
        tests = (golden["sum_neighbors"] - n) // 2 if dom == "main" else golden["sum_min_neighbors_minpts"]
        ops = tests * pred_ops(d)
        ach = ops / (ms / 1e3) / 1e12
        out = {"bound": "alu", "achieved": round(ach, 3), "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
               "frac": round(ach / ALU_PEAK_TOPS, 4), "frac_vs_packed_peak": round(ach / ALU_PEAK_PACKED_TOPS, 4),
               "kernel": single[dom], "stage": dom, "ms": round(ms, 4),
               "work": f"{tests} neighbour tests x {pred_ops(d)} fp32 ops"}
        pipeline["t_roof_alu_ms"] = round(ops / (ALU_PEAK_TOPS * 1e12) * 1e3, 4)
    else:
        b = sb.get(dom, 0)
        ach = b / (ms / 1e3) / 1e9
        out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": single[dom], "stage": dom, "ms": round(ms, 4),
               "alg_bytes": int(b)}
    t = (traffic_db or {}).get(f"{algo}:{dom}")
    out["traffic"] = t["bytes"] if t else None  # HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)
    out["traffic_detail"] = t
    return out, pipeline


def source_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2103_05162_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE), scaled by a
    copy-kernel calibration; only valid while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    db = json.load(open(path))
    if db.get("src_hash") != source_hash():
        return None
    return db.get("kernels")


def load_golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    return json.load(open(path)) if os.path.exists(path) else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(points, eps, min_pts, frac):
    """The oracle on a spatial window of the headline workload (all usable cores)."""
    import oracle
    from workloads.gen import window
    sample = window(points, frac)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    oracle.dbscan(sample, eps, min_pts, threads=cores)
    t = time.perf_counter() - t0
    return {"value": round(sample.shape[0] / t / 1e6, 4), "unit": "Mpts/s", "cores": cores, "kind": "oracle",
            "sample": f"window, not the whole set: the {sample.shape[0]} points inside the corner box holding "
                      f"{frac:.4g} of the bounding volume (same local density), clustered in {t:.2f} s",
            "cpu_model": cpu_model()}


def cpu_full(names, cores):
    """The oracle on whole small workloads, at every usable core and at one thread."""
    import oracle
    from workloads.gen import workload
    out = {}
    for name in names:
        w = workload(name)
        row = {"n": w.n, "cpu_model": cpu_model()}
        for th in (cores, 1):
            t0 = time.perf_counter()
            oracle.dbscan(w.points, w.eps, w.min_pts, threads=th)
            t = time.perf_counter() - t0
            row[f"threads_{th}"] = {"s": round(t, 3), "mpts_per_s": round(w.n / t / 1e6, 4)}
            log(f"[bench] cpu oracle {name} at {th} threads: {t:.2f} s")
        out[name] = row
    return out


def main():
    args = parse()
    if args.gpus != 1:
        log(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
            "the method here is single-device and no multi-GPU path is built.")
        sys.exit(2)
    import torch
    import paper_2103_05162_amd as fdb

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib:
        # kernels of known traffic for reading HBM counters: a streaming copy, then a
        # gather of 12-byte rows (the shape of the gather to key order) through an
        # identity index and through a random permutation of the same size
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        rows = src[: nel // 3 * 3].view(-1, 3)
        ident = torch.arange(rows.shape[0], device=dev)
        perm = torch.randperm(rows.shape[0], device=dev, generator=torch.Generator(device=dev).manual_seed(1))
        torch.index_select(rows, 0, ident)
        torch.index_select(rows, 0, perm)
        torch.cuda.synchronize()
        log(f"[bench] calibration kernels done: copy of {args.copy_calibration_mib} MiB, gathers of "
            f"{rows.shape[0]} 12-byte rows by identity and by a random permutation")
        del src, dst, rows, ident, perm
    h = fdb.Handle(0)
    algos = ["densebox", "fdbscan"] if args.algo == "both" else [args.algo]
    head = algos[0]
    c3 = run_leg(fdb, h, "c3_dense3d_8m", algos, args.steps, args.warmup, args.scale, tune=args.tune)
    r = c3["algos"][head]
    ms = r["ms_per_step"]
    if args.scale == 1.0 and r["labels_match_oracle_golden"] is False:
        log(f"[bench] WARNING: {head} labels differ from the oracle's golden hashes")
    out = {
        "metric": "Mpts/s clustered (3D, 8M pts)",
        "value": r["mpts_per_s"],
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c3['workload']}: {c3['n']} 3D float32 points, 500 Gaussian clumps (sigma 5e-4, "
                               f"80%) + uniform background, eps={c3['eps']:g}, minPts={c3['min_pts']}",
                   "algo": head, "num_clusters": r["num_clusters"]},
        "roofline": r["roofline"],
        "pipeline_roofline": r["pipeline"],
        "legs": {"c3_dense3d_8m": c3},
        "src_hash": source_hash(),
    }
    if not args.no_small_legs and args.scale == 1.0:
        for name in ("c2_fof3d_2m", "c1_blobs2d_16k"):
            out["legs"][name] = run_leg(fdb, h, name, ["densebox", "fdbscan"], args.steps, args.warmup,
                                        tune=args.tune and name == "c2_fof3d_2m")
    torch.cuda.empty_cache()
    if args.batched_algo != "none":
        log(f"[bench] batched leg ({args.batched_algo})")
        b = time_batched(fdb, h, args.batched_algo, args.steps, args.warmup, args.clouds, args.loop_passes,
                         int(args.ooc_budget_gib * (1 << 30)), tune=args.tune)
        log(f"[bench] batched: {b['ms']:.2f} ms per batch, graph replay {b['graph_ms']:.2f} ms, "
            f"loop {b['loop_ms']} ms, identical={b['identical']}, oracle: {b['golden']}")
        for st, v in sorted(b["stages"].items(), key=lambda kv: -kv[1]):
            log(f"    {st:12s} {v:9.3f} ms")
        out["batched"] = {
            "workload": f"{args.clouds} 3D clouds of 1024-65535 points (log-uniform), 1-20 clumps each, "
                        f"eps 0.005-0.02 per cloud, minPts 5; {b['n']} points",
            "algo": args.batched_algo, "ms_per_batch": round(b["ms"], 3),
            "clouds_per_s": round(args.clouds / (b["ms"] / 1e3), 1),
            "mpts_per_s": round(b["n"] / (b["ms"] / 1e3) / 1e6, 3),
            "graph_replay_ms_per_batch": round(b["graph_ms"], 3),
            "graph_replay_clouds_per_s": round(args.clouds / (b["graph_ms"] / 1e3), 1),
            "graph_replay_identical": b["graph_identical"],
            "loop_ms": round(b["loop_ms"], 3) if b["loop_ms"] else None,
            "loop_clouds_per_s": round(args.clouds / (b["loop_ms"] / 1e3), 1) if b["loop_ms"] else None,
            "speedup_vs_loop": round(b["loop_ms"] / b["ms"], 3) if b["loop_ms"] else None,
            "identical_to_loop": b["identical"], "oracle_golden": b["golden"], "clusters": b["clusters"],
            "info": b["info"], "tuned": b["tuned"],
            "stages_ms": {k2: round(v, 4) for k2, v in b["stages"].items()}}
        if b["ooc"]:
            o = b["ooc"]
            log(f"[bench] out-of-core: {o['ms']:.2f} ms per batch in {o['budget'] >> 20} MiB, identical={o['identical']}")
            out["batched"]["out_of_core"] = {
                "workload": "the same batch in pinned host memory, clustered in groups of whole clouds inside a "
                            "device budget below what the batch needs (host-to-device and back included)",
                "device_budget_gib": round(o["budget"] / (1 << 30), 3),
                "device_bytes_in_core_gib": round(o["need"] / (1 << 30), 3),
                "ms_per_batch": round(o["ms"], 3), "clouds_per_s": round(args.clouds / (o["ms"] / 1e3), 1),
                "mpts_per_s": round(b["n"] / (o["ms"] / 1e3) / 1e6, 3),
                "identical_to_in_core": o["identical"]}
    if args.served_algo != "none":
        log(f"[bench] served leg ({args.served_algo})")
        rates = [args.rate] + [x for x in args.extra_rates if x != args.rate]
        out["served"] = time_served(fdb, args.served_algo, args.requests, rates, args.budget_gib,
                                    args.pool_per_dim)
    if not args.no_cpu_baseline:
        from workloads.gen import workload
        w = workload("c3_dense3d_8m", args.scale)
        log(f"[bench] cpu oracle on a {args.cpu_window:g} window of the headline set")
        out["cpu_baseline"] = cpu_baseline(w.points, w.eps, w.min_pts, args.cpu_window)
        if args.scale == 1.0 and not args.no_small_legs:
            out["cpu_oracle_full"] = cpu_full(["c1_blobs2d_16k", "c2_fof3d_2m"], len(os.sched_getaffinity(0)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
