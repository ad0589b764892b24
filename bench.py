#!/usr/bin/env python3
"""Benchmark: DBSCAN throughput on one MI355X.

One step = one full clustering of the workload (every stage from device-resident
float32 points to device-resident int32 labels: bounds, keys, sort, gather,
LBVH, core pass, fused union traversal, finalisation, canonical ids, border pass,
scatter). The workload is the dense-clump 3D set: 8,388,608 points, 500 clumps
of sigma 5e-4 holding 80% of them, uniform background, eps = 0.002, minPts = 10.
DenseBox is the headline algorithm; FDbscan is measured beside it.

A second leg clusters a batch of 4096 uneven 3D clouds (1024-65535 points each,
every cloud with its own eps) in one call and reports clouds/s beside a loop of
one call per cloud over the same data, and whether both give identical labels.

A third leg replays an open-loop request stream (Poisson arrivals, clouds of
10k-2M points, 2D and 3D, mixed eps and minPts) against the continuous-batching
server and against a plain one-job-at-a-time server, and reports p50/p99
latency, throughput and whether each keeps up.

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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
# fp32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s for the plain
# (non-packed, non-fused) v_sub/v_mul/v_add/v_cmp the neighbour test compiles to; packed
# fp32 would double it (78.6 T) but is disabled in this build. The published 157.3 TFLOP/s
# counts a packed FMA as 4 flops.
ALU_PEAK_TOPS = 39.3
PRED_OPS_3D = 9         # 3 sub, 3 mul, 2 add, 1 compare per neighbour test

P_BYTES = 12            # one 3D float32 point
NODE_BYTES = 36         # internal node: box + range end + split (32 B) + escape link (4 B)
I_BYTES, F_BYTES = 4, 1


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
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--batched-algo", default="densebox", choices=["none", "densebox", "fdbscan"],
                    help="algorithm of the batched many-cloud leg (none = skip it)")
    ap.add_argument("--clouds", type=int, default=4096, help="clouds in the batched leg")
    ap.add_argument("--loop-passes", type=int, default=1,
                    help="timed passes of the one-call-per-cloud loop beside the batch (0 = skip it)")
    ap.add_argument("--served-algo", default="densebox", choices=["none", "densebox", "fdbscan"],
                    help="algorithm of the served leg (none = skip it)")
    ap.add_argument("--requests", type=int, default=22000, help="requests in the served trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="request arrivals per second")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="HBM budget of the served batches")
    ap.add_argument("--pool-per-dim", type=int, default=32, help="resident clouds per dimension")
    ap.add_argument("--ooc-budget-gib", type=float, default=6.0,
                    help="device budget of the out-of-core batched leg (0 = skip it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (PMC calibration)")
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
    return dict(ms=ms, k=k, stages=per_call, info=h.last_info(), sizes=h.last_counts())


def time_batched(fdb, h, algo, steps, warmup, num_clouds, loop_passes, ooc_budget=0):
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

    if loop_passes <= 0:
        return dict(ms=ms, loop_ms=None, n=n, identical=None, info=info, ooc=ooc,
                    stages={k2: v / max(calls, 1) for k2, v in stages.items()}, clusters=int(ncl.sum().item()))
    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_passes):
        loop()
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3 / loop_passes
    same = bool(torch.equal(labels, lab2) and torch.equal(core, core2))
    return dict(ms=ms, loop_ms=loop_ms, n=n, identical=same, info=info, ooc=ooc,
                stages={k2: v / max(calls, 1) for k2, v in stages.items()},
                clusters=int(ncl.sum().item()))


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


def time_served(fdb, algo, requests, rate, budget_gib, pool_per_dim, warm_s=1.0):
    """Served leg: the same open-loop trace replayed on the continuous-batching server
    and on the plain one-job-at-a-time server; every request's labels must agree."""
    import torch
    from workloads.gen import served_trace
    t0 = time.perf_counter()
    pool, req = served_trace(requests=requests, rate=rate, pool_per_dim=pool_per_dim)
    log(f"[bench] served trace: {requests} requests at {rate:g}/s, pool of {2 * pool_per_dim} clouds "
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
    res = {}
    rng = np.random.default_rng(0)
    first = int(np.searchsorted(req["arrival_s"], warm_s))
    sample = rng.choice(np.arange(first, requests), size=min(64, requests - first), replace=False)
    kept = {}
    for mode in ("batched", "fifo"):
        log(f"[bench] serving the trace ({mode})")
        res[mode] = replay(fdb, mode, algo, budget, 4096, ptrs, req, out, warm_s)
        log(f"[bench]   {mode}: {res[mode]}")
        got = {int(r): out[int(req['out_off'][r]):int(req['out_off'][r]) + int(req['n'][r])].cpu() for r in sample}
        kept[mode] = got
    same = all(torch.equal(kept["batched"][r], kept["fifo"][r]) for r in kept["batched"])
    del out, pool_dev
    torch.cuda.empty_cache()
    return {"workload": f"{requests} requests, Poisson arrivals at {rate:g}/s (first {warm_s:g} s not counted), "
                        f"sizes log-uniform 10240-2097151 from a pool of {2 * pool_per_dim} clouds, d in {{2,3}}, "
                        f"minPts in {{2,5,10}}, eps 0.005-0.02",
            "algo": algo, "hbm_budget_gib": budget_gib, "mean_points": round(float(req["n"].mean()), 1),
            "batched": res["batched"], "fifo": res["fifo"],
            "p99_speedup_vs_fifo": round(res["fifo"]["p99_ms"] / res["batched"]["p99_ms"], 3)
            if res["batched"]["p99_ms"] > 0 else None,
            "identical_labels_sampled": same, "sampled_requests": len(sample)}


def algorithmic_bytes(stage, n, sizes):
    """Compulsory HBM bytes of one launch of a single-kernel stage: every input read
    once and every output written once (cache reuse is free)."""
    m = sizes["prims"]                      # BVH primitives
    c = sizes["dense_cells"]
    ns = m - c if c else n                  # points outside dense cells (all points for FDbscan)
    tree = max(m - 1, 0) * NODE_BYTES + m * I_BYTES                 # nodes + leaf escape links
    prims = m * (2 * I_BYTES) + c * 32 if c else 0                  # DenseBox primitive records
    pts = n * P_BYTES                                               # every point once
    if stage == "core":        # queries (points outside dense cells) count neighbours, write a flag
        return pts + tree + prims + ns * F_BYTES
    if stage == "main_points":  # queries read flag + label, candidates' flags and labels, label writes
        return pts + tree + prims + n * (F_BYTES + I_BYTES) + ns * I_BYTES
    if stage == "main_cells":  # dense-cell queries
        return pts + tree + prims + n * (F_BYTES + I_BYTES) + c * I_BYTES
    if stage == "main":        # FDbscan fused traversal
        return pts + tree + n * (F_BYTES + I_BYTES) + n * I_BYTES
    if stage == "border":      # non-core queries: candidates' flags, labels and cluster ids
        return pts + tree + prims + n * (F_BYTES + 2 * I_BYTES) + ns * I_BYTES
    if stage == "scatter":     # labels, flags, permutation, ids in; labels + flags out
        return n * (I_BYTES + F_BYTES + I_BYTES + I_BYTES + I_BYTES) + n * (I_BYTES + F_BYTES)
    if stage == "finalize":
        return n * 2 * I_BYTES
    return None


def roofline(algo, stages, n, sizes, golden, traffic_db):
    single = ["core", "main", "main_cells", "main_points", "border", "scatter", "finalize"]
    cand = {k: v for k, v in stages.items() if k in single}
    if not cand:
        return None
    # DenseBox: the isolated-point test settles part of the core queries before the
    # walks; the two stages together do the core pass the byte count describes
    core_parts = ["isolated", "core"] if "core" in cand and "isolated" in stages else ["core"]
    if len(core_parts) == 2:
        cand["core"] = cand["core"] + stages["isolated"]
    dom = max(cand, key=cand.get)
    ms = cand[dom]
    if algo == "fdbscan" and dom in ("main", "core") and golden and "sum_neighbors" in golden:
        # ALU bound: one neighbour test per pair (each pair once in the masked main phase;
        # up to minPts tests per point in the core phase)
        tests = (golden["sum_neighbors"] - n) // 2 if dom == "main" else golden["sum_min_neighbors_minpts"]
        ach = tests * PRED_OPS_3D / (ms / 1e3) / 1e12
        out = {"bound": "alu", "achieved": round(ach, 3), "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
               "frac": round(ach / ALU_PEAK_TOPS, 4), "kernel": dom, "ms": round(ms, 4),
               "work": f"{tests} neighbour tests x {PRED_OPS_3D} fp32 ops"}
    else:
        b = algorithmic_bytes(dom, n, sizes)
        ach = b / (ms / 1e3) / 1e9
        out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": dom, "ms": round(ms, 4), "alg_bytes": b}
        if dom == "core":
            out["stages"] = core_parts
    t = (traffic_db or {}).get(f"{algo}:{dom}")
    out["traffic"] = t["bytes"] if t else None  # HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)
    out["traffic_detail"] = t
    return out


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
    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst
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
    golden = load_golden("c3_dense3d_8m") if args.scale == 1.0 else None
    traffic_db = load_traffic()
    for a in algos:
        res[a]["roofline"] = roofline(a, res[a]["stages"], w.n, res[a]["sizes"], golden, traffic_db)
    if golden is not None:
        for a in algos:
            if res[a]["k"] != golden["num_clusters"]:
                log(f"[bench] WARNING: {a} K={res[a]['k']} but the oracle's K={golden['num_clusters']}")
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
        "roofline": res[head]["roofline"],
        "stages_ms": {a: {k2: round(v, 4) for k2, v in res[a]["stages"].items()} for a in algos},
        "per_algo": {a: {"ms_per_step": round(res[a]["ms"], 4),
                         "mpts_per_s": round(w.n / (res[a]["ms"] / 1e3) / 1e6, 3),
                         "mfeatures_per_s": round(3 * w.n / (res[a]["ms"] / 1e3) / 1e6, 3),
                         "num_clusters": res[a]["k"], "sizes": res[a]["sizes"],
                         "roofline": res[a]["roofline"]} for a in algos},
        "src_hash": source_hash(),
    }
    if args.batched_algo != "none":
        del pts
        torch.cuda.empty_cache()
        log(f"[bench] batched leg ({args.batched_algo})")
        b = time_batched(fdb, h, args.batched_algo, args.steps, args.warmup, args.clouds, args.loop_passes,
                         int(args.ooc_budget_gib * (1 << 30)))
        log(f"[bench] batched: {b['ms']:.2f} ms per batch, loop {b['loop_ms']} ms, identical={b['identical']}")
        for st, v in sorted(b["stages"].items(), key=lambda kv: -kv[1]):
            log(f"    {st:12s} {v:9.3f} ms")
        out["batched"] = {
            "workload": f"{args.clouds} 3D clouds of 1024-65535 points (log-uniform), 1-20 clumps each, "
                        f"eps 0.005-0.02 per cloud, minPts 5; {b['n']} points",
            "algo": args.batched_algo, "ms_per_batch": round(b["ms"], 3),
            "clouds_per_s": round(args.clouds / (b["ms"] / 1e3), 1),
            "mpts_per_s": round(b["n"] / (b["ms"] / 1e3) / 1e6, 3),
            "loop_ms": round(b["loop_ms"], 3) if b["loop_ms"] else None,
            "loop_clouds_per_s": round(args.clouds / (b["loop_ms"] / 1e3), 1) if b["loop_ms"] else None,
            "speedup_vs_loop": round(b["loop_ms"] / b["ms"], 3) if b["loop_ms"] else None,
            "identical_to_loop": b["identical"], "clusters": b["clusters"], "info": b["info"],
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
        out["served"] = time_served(fdb, args.served_algo, args.requests, args.rate, args.budget_gib,
                                    args.pool_per_dim)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu oracle on a {args.cpu_window:g} window")
        out["cpu_baseline"] = cpu_baseline(w.points, w.eps, w.min_pts, args.cpu_window)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
