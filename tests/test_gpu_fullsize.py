"""Parity at the configured full sizes, in the launch configuration bench.py
times (default options, one call on cuda:0).

Two independent checks per workload and algorithm:
  * the whole output against the oracle's full-size run, stored by
    tests/golden/make_golden.py (which calls only the oracle): SHA-256 of the
    canonical labels and core flags, K, core and noise counts;
  * sampled outputs the oracle computes one by one by brute force over all
    points: core flags, and for sampled points the labels of their core
    neighbours (a core point shares its label with every core neighbour; a
    non-core point carries the smallest label among its core neighbours, or -1).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from workloads.gen import workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALGOS = ["fdbscan", "densebox"]
SAMPLES = 48


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2103_05162_amd as fdb
    fdb.load()
    return torch.device("cuda:0")


_cache = {}


def _run(dev, name, algo):
    key = (name, algo)
    if key not in _cache:
        import torch
        import paper_2103_05162_amd as fdb
        w = workload(name)
        _say(f"[gpu] full-size {name} n={w.n} algo={algo}")
        t = torch.from_numpy(w.points).to(dev)
        labels, core, k = fdb.dbscan(t, w.eps, w.min_pts, algo=algo)
        torch.cuda.synchronize()
        info = fdb.default_handle(0).last_info()
        _cache[key] = (w, labels.cpu().numpy(), core.cpu().numpy(), k, info)
        del t
    return _cache[key]


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no golden values for {name}")
    return json.load(open(path))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name", ["c2_fof3d_2m", "c3_dense3d_8m"])
def test_full_size_matches_oracle_golden(dev, name, algo):
    g = _golden(name)
    w, labels, core, k, info = _run(dev, name, algo)
    assert info == 0
    assert hashlib.sha256(w.points.astype("<f4").tobytes()).hexdigest() == g["points_sha256"], \
        "generator output differs from the one the golden values were made from"
    assert k == g["num_clusters"]
    assert int(core.sum()) == g["num_core"]
    assert int((labels < 0).sum()) == g["num_noise"]
    assert hashlib.sha256(core.astype(np.uint8).tobytes()).hexdigest() == g["core_sha256"]
    assert hashlib.sha256(labels.astype("<i4").tobytes()).hexdigest() == g["labels_sha256"]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name", ["c2_fof3d_2m", "c3_dense3d_8m"])
def test_full_size_sampled_brute_force(dev, name, algo):
    w, labels, core, k, info = _run(dev, name, algo)
    rng = np.random.default_rng(7)
    # half the samples at random, half among non-core points (the rarer case)
    noncore = np.flatnonzero(~core)
    idx = np.concatenate([rng.choice(w.n, SAMPLES // 2, replace=False),
                          rng.choice(noncore, min(SAMPLES // 2, noncore.size), replace=False)])
    assert labels.min() >= -1 and labels.max() == k - 1
    for i in idx:
        nb = oracle.neighbors_of(w.points, w.eps, int(i))
        assert core[i] == (len(nb) >= w.min_pts), f"core flag of point {i}"
        core_nb = nb[core[nb]]
        if core[i]:
            assert np.all(labels[core_nb] == labels[i]), f"core point {i} split from a core neighbour"
        else:
            want = labels[core_nb].min() if core_nb.size else -1
            assert labels[i] == want, f"non-core point {i}: {labels[i]} != {want}"


def test_full_batch_matches_oracle_golden(dev):
    """The 4096-cloud batch at its configured size, in the bench's launch
    configuration: every cloud's K and the SHA-256 of its canonical labels and core
    flags against the oracle's cloud-by-cloud run."""
    import torch
    import paper_2103_05162_amd as fdb
    from workloads.gen import batched_clouds
    g = _golden("c4_batched_4096")
    clouds, eps, mp = batched_clouds(g["num_clouds"])
    assert hashlib.sha256(eps.astype("<f4").tobytes()).hexdigest() == g["eps_sha256"]
    assert hashlib.sha256(clouds[0].astype("<f4").tobytes()).hexdigest() == g["points_sha256_first_cloud"]
    offs = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    assert int(offs[-1]) == g["n"]
    pts = torch.from_numpy(np.concatenate(clouds)).to(dev)
    del clouds
    d_off, d_eps, d_mp = (torch.from_numpy(a).to(dev) for a in (offs, eps, mp))
    _say(f"[gpu] full batch: {g['num_clouds']} clouds, {g['n']} points")
    lab, core, k = fdb.dbscan_batched(pts, d_off, d_eps, d_mp, algo="densebox")
    torch.cuda.synchronize()
    assert fdb.default_handle(0).last_info() == 0
    lab, core, k = lab.cpu().numpy(), core.cpu().numpy().astype(np.uint8), k.cpu().numpy()
    bad = []
    for c, (kc, ls, cs) in enumerate(g["clouds"]):
        sl = slice(int(offs[c]), int(offs[c + 1]))
        if (int(k[c]) != kc or hashlib.sha256(lab[sl].astype("<i4").tobytes()).hexdigest()[:16] != ls
                or hashlib.sha256(core[sl].tobytes()).hexdigest()[:16] != cs):
            bad.append(c)
    assert not bad, f"clouds differing from the oracle: {bad[:10]} ({len(bad)} of {len(g['clouds'])})"


def test_served_requests_match_oracle_golden(dev):
    """A fixed sample of the served trace's requests, submitted to the
    continuous-batching server together with their neighbours in the trace (so they
    share batches with other jobs): labels and K against the oracle's hashes."""
    import torch
    import paper_2103_05162_amd as fdb
    from workloads.gen import served_trace
    g = _golden("c5_served_sample")
    t = g["trace"]
    pool, req = served_trace(requests=t["requests"], rate=t["rate"], pool_per_dim=t["pool_per_dim"])
    want = {int(e[0]): e for e in g["requests"]}
    # each sampled request with the two requests after it in the trace
    jobs = sorted({r + d for r in want for d in (0, 1, 2) if r + d < len(req["n"])})
    dev_pool = {}
    srv = fdb.Server(0, budget_bytes=16 << 30, max_batch=4096, mode="batched", algo="densebox")
    outs, tickets = {}, {}
    try:
        for r in jobs:
            d, c = int(req["dim"][r]), int(req["cloud"][r])
            if (d, c) not in dev_pool:
                dev_pool[(d, c)] = torch.from_numpy(pool[d][c]).to(dev)
            n = int(req["n"][r])
            outs[r] = torch.full((n,), -7, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        _say(f"[gpu] served sample: {len(want)} requests in {len(jobs)} jobs")
        for r in jobs:
            d, c = int(req["dim"][r]), int(req["cloud"][r])
            tickets[r] = srv.submit_raw(dev_pool[(d, c)].data_ptr(), int(req["n"][r]), d, float(req["eps"][r]),
                                        int(req["min_pts"][r]), outs[r].data_ptr())
        srv.drain()
        res = {r: srv.poll(tickets[r]) for r in want}
    finally:
        srv.close()
    bad = []
    for r, e in want.items():
        _, d, c, n, kc, ls, _cs = e
        assert int(req["n"][r]) == n and int(req["dim"][r]) == d and int(req["cloud"][r]) == c
        got = outs[r].cpu().numpy().astype("<i4")
        if res[r]["num_clusters"] != kc or hashlib.sha256(got.tobytes()).hexdigest()[:16] != ls:
            bad.append(r)
    assert not bad, f"requests differing from the oracle: {bad}"
