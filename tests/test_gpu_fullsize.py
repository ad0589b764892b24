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
