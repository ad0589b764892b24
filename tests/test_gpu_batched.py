"""Batched clustering (many independent clouds in one launch sequence) against
per-cloud calls and the oracle: every cloud's canonical labels, core flags and
K must equal those of the cloud clustered alone."""
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import assert_tolerance_mode
from workloads.gen import batched_clouds

pytestmark = pytest.mark.gpu
ALGOS = ["fdbscan", "densebox"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2103_05162_amd as fdb
    fdb.load()
    return torch.device("cuda:0")


def _random_batch(seed, dim, num):
    rng = np.random.default_rng(seed)
    clouds, eps, mp = [], [], []
    for c in range(num):
        kind = rng.integers(0, 6)
        n = int([0, 1, 2, rng.integers(3, 200), rng.integers(200, 3000), rng.integers(3000, 9000)][kind])
        k = int(rng.integers(1, 6))
        cen = rng.uniform(0, 1, size=(k, dim))
        lab = rng.integers(0, k, size=n)
        pts = cen[lab] + rng.uniform(0.003, 0.03) * rng.standard_normal((n, dim))
        noise = rng.random(n) < 0.2
        pts[noise] = rng.uniform(0, 1, size=(int(noise.sum()), dim))
        clouds.append(pts.astype(np.float32))
        eps.append(float(np.float32(rng.uniform(0.005, 0.04))))
        mp.append(int(rng.choice([1, 2, 3, 5, 10])))
    return clouds, np.asarray(eps, np.float32), np.asarray(mp, np.int32)


def _run_batch(dev, clouds, eps, mp, algo, border="canonical"):
    import torch
    import paper_2103_05162_amd as fdb
    sizes = [len(c) for c in clouds]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    dim = clouds[0].shape[1] if clouds else 3
    allp = np.concatenate(clouds) if sum(sizes) else np.zeros((0, dim), np.float32)
    t = torch.from_numpy(np.ascontiguousarray(allp)).to(dev)
    labels, core, k = fdb.dbscan_batched(t, torch.from_numpy(offs).to(dev), torch.from_numpy(eps).to(dev),
                                         torch.from_numpy(mp).to(dev), algo=algo, border=border)
    torch.cuda.synchronize()
    info = fdb.default_handle(0).last_info()
    return offs, labels.cpu().numpy(), core.cpu().numpy(), k.cpu().numpy(), info


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("dim,seed", [(3, 1), (2, 2)])
def test_batch_equals_each_cloud_alone(dev, algo, dim, seed):
    clouds, eps, mp = _random_batch(seed, dim, 60)
    _say(f"[gpu] batch of {len(clouds)} clouds, {sum(map(len, clouds))} points, d={dim}, {algo}")
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo)
    assert info == 0
    for c, pts in enumerate(clouds):
        rl, rc, rk = oracle.dbscan(pts, float(eps[c]), int(mp[c]))
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == rk, (c, len(pts), k[c], rk)
        assert np.array_equal(core[sl], rc), c
        assert np.array_equal(labels[sl], rl), c


@pytest.mark.parametrize("algo", ALGOS)
def test_batch_first_claim_mode(dev, algo):
    clouds, eps, mp = _random_batch(3, 3, 30)
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo, border="first")
    assert info == 0
    for c, pts in enumerate(clouds):
        if len(pts) == 0:
            continue
        rl, rc, rk = oracle.dbscan(pts, float(eps[c]), int(mp[c]))
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == rk
        assert_tolerance_mode(pts, float(eps[c]), labels[sl], core[sl], rl, rc, oracle.check_border)


@pytest.mark.parametrize("algo", ALGOS)
def test_many_uneven_clouds_match_single_calls(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    clouds, eps, mp = batched_clouds(num_clouds=96, lo=1024, hi=16384)
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo)
    assert info == 0
    for c, pts in enumerate(clouds):
        t = torch.from_numpy(pts).to(dev)
        l1, c1, k1 = fdb.dbscan(t, float(eps[c]), int(mp[c]), algo=algo)
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == k1
        assert np.array_equal(labels[sl], l1.cpu().numpy()) and np.array_equal(core[sl], c1.cpu().numpy())


def _check_others(clouds, eps, mp, offs, labels, core, k, skip):
    for c, pts in enumerate(clouds):
        if c in skip:
            continue
        rl, rc, rk = oracle.dbscan(pts, float(eps[c]), int(mp[c]))
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == rk and np.array_equal(core[sl], rc) and np.array_equal(labels[sl], rl), c


@pytest.mark.parametrize("algo", ALGOS)
def test_bad_cloud_parameters_are_reported(dev, algo):
    import paper_2103_05162_amd as fdb
    clouds, eps, mp = _random_batch(4, 3, 6)
    clouds = [c if len(c) else np.zeros((5, 3), np.float32) for c in clouds]
    eps[2] = -1.0
    mp[4] = 0
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo)
    assert info & fdb.FDB_INFO_BAD_PARAMS
    assert not info & fdb.FDB_INFO_NONFINITE
    assert k[2] == -1 and k[4] == -1
    _check_others(clouds, eps, mp, offs, labels, core, k, {2, 4})


@pytest.mark.parametrize("algo", ALGOS)
def test_nonfinite_cloud_is_isolated(dev, algo):
    import paper_2103_05162_amd as fdb
    clouds, eps, mp = _random_batch(5, 3, 6)
    clouds = [c if len(c) > 3 else np.zeros((5, 3), np.float32) for c in clouds]
    clouds[1][0, 2] = np.nan
    clouds[3][-1, 0] = np.inf
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo)
    assert info & fdb.FDB_INFO_NONFINITE
    assert not info & fdb.FDB_INFO_INTERNAL
    assert k[1] == -1 and k[3] == -1
    _check_others(clouds, eps, mp, offs, labels, core, k, {1, 3})


def test_empty_batch(dev):
    import torch
    import paper_2103_05162_amd as fdb
    t = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    offs = torch.zeros(4, dtype=torch.int64, device=dev)
    labels, core, k = fdb.dbscan_batched(t, offs, torch.full((3,), 0.1, device=dev),
                                         torch.full((3,), 3, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    assert k.cpu().tolist() == [0, 0, 0]


@pytest.mark.parametrize("algo", ALGOS)
def test_batch_dbscan_star(dev, algo):
    clouds, eps, mp = _random_batch(6, 3, 40)
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, algo, border="none")
    assert info == 0
    for c, pts in enumerate(clouds):
        rl, rc, rk = oracle.dbscan_star(pts, float(eps[c]), int(mp[c]))
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == rk and np.array_equal(core[sl], rc) and np.array_equal(labels[sl], rl), c


_LANE = {}


def _lane_batch():
    """~150 clouds of tight 6-point clumps: more than 65,536 dense cells in the
    batch as a whole, so the dense-cell main phase takes one lane per cell."""
    if not _LANE:
        rng = np.random.default_rng(93)
        clouds, eps, mp = [], [], []
        for c in range(150):
            k = int(rng.integers(550, 750))
            cen = rng.uniform(0, 1, size=(k, 3))
            pts = np.repeat(cen, 6, axis=0) + 1e-4 * rng.standard_normal((k * 6, 3))
            noise = rng.uniform(0, 1, size=(int(rng.integers(0, 300)), 3))
            pts = np.concatenate([pts, noise])[rng.permutation(k * 6 + len(noise))]
            clouds.append(pts.astype(np.float32))
            eps.append(float(np.float32(rng.uniform(0.002, 0.004))))
            mp.append(int(rng.choice([3, 4, 6])))
        _LANE["case"] = (clouds, np.asarray(eps, np.float32), np.asarray(mp, np.int32))
    return _LANE["case"]


@pytest.mark.parametrize("border", ["canonical", "first", "none"])
def test_batch_lane_per_cell_kernel_matches_oracle(dev, border):
    import paper_2103_05162_amd as fdb
    clouds, eps, mp = _lane_batch()
    _say(f"[gpu] lane-per-cell batch: {len(clouds)} clouds, {sum(map(len, clouds))} points ({border})")
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, "densebox", border=border)
    assert info == 0
    assert fdb.default_handle(0).last_counts()["dense_cells"] > 65536
    for c, pts in enumerate(clouds):
        sl = slice(offs[c], offs[c + 1])
        if border == "none":
            rl, rc, rk = oracle.dbscan_star(pts, float(eps[c]), int(mp[c]))
        else:
            rl, rc, rk = oracle.dbscan(pts, float(eps[c]), int(mp[c]))
        assert k[c] == rk, (c, k[c], rk)
        if border == "first":
            assert_tolerance_mode(pts, float(eps[c]), labels[sl], core[sl], rl, rc, oracle.check_border)
        else:
            assert np.array_equal(core[sl], rc) and np.array_equal(labels[sl], rl), c


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_cloud_wider_than_the_key_range(dev, dim):
    """A cloud whose extent over the DenseBox cell side exceeds the key bits a
    batch leaves per axis (its cell coordinates are clamped at the top): clumps
    near the origin and far out, all clustered as the oracle does."""
    rng = np.random.default_rng(94 + dim)
    clouds, eps, mp = [], [], []
    for c in range(5):
        pts = rng.uniform(0, 1, size=(800, dim)) * 0.2
        pts = np.concatenate([pts, 0.1 + 0.003 * rng.standard_normal((400, dim))])
        clouds.append(pts.astype(np.float32))
        eps.append(0.01)
        mp.append(4)
    # bits per axis below the cloud id: floor((64 - ceil(log2 5)) / d), at most 21 (3D) / 31 (2D)
    bpd = min(21 if dim == 3 else 31, (64 - 3) // dim)
    far = 1.5 * (2 ** bpd) * 0.01 / np.sqrt(dim)   # beyond the last key cell on every axis
    wide = np.concatenate([0.003 * rng.standard_normal((300, dim)),
                           far + 0.003 * rng.standard_normal((300, dim)),
                           1.3 * far + 0.003 * rng.standard_normal((300, dim)),
                           far * rng.uniform(0, 1.3, size=(200, dim))]).astype(np.float32)
    clouds[2] = wide[rng.permutation(len(wide))]
    eps, mp = np.asarray(eps, np.float32), np.asarray(mp, np.int32)
    offs, labels, core, k, info = _run_batch(dev, clouds, eps, mp, "densebox")
    assert info == 0
    for c, pts in enumerate(clouds):
        rl, rc, rk = oracle.dbscan(pts, float(eps[c]), int(mp[c]))
        sl = slice(offs[c], offs[c + 1])
        assert k[c] == rk and np.array_equal(core[sl], rc) and np.array_equal(labels[sl], rl), c
    rl, rc, rk = oracle.dbscan(clouds[2], float(eps[2]), int(mp[2]))
    assert rk >= 3 and rc.sum() > 600
