"""The union-find forest check (FDB_FLAG_VALIDATE, fdb_debug_forest) on one GPU.

The fused main phase (Section 3.2's union and claim steps) keeps a forest in
which a core point's parent is a core point of smaller index and every other
point points at itself or at a core point. The check is pinned by hand-built
forests with a known number of violations, then run after the main phase of
real calls, where it must find none.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads.gen import batched_clouds, workload

pytestmark = pytest.mark.gpu


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


def _forest_bad(dev, parent, core):
    import torch
    import paper_2103_05162_amd as fdb
    h = fdb.default_handle(0)
    p = torch.from_numpy(np.asarray(parent, np.int32)).to(dev)
    c = torch.from_numpy(np.asarray(core, np.uint8)).to(dev) if core is not None else None
    return h.debug_forest(p.data_ptr(), c.data_ptr() if c is not None else None, len(parent))


def test_hand_built_forests_count_each_violation_once(dev):
    # a valid forest: cores 0..3 under 0, non-core 4 claimed by core 2, non-core 5 alone
    parent = [0, 0, 1, 0, 2, 5]
    core = [1, 1, 1, 1, 0, 0]
    assert _forest_bad(dev, parent, core) == 0
    # a core pointing at a larger index
    assert _forest_bad(dev, [0, 3, 1, 3, 2, 5], core) == 1
    # a core pointing at a non-core point
    assert _forest_bad(dev, [0, 0, 4, 0, 2, 5], core) == 1
    # a non-core point pointing at a non-core point
    assert _forest_bad(dev, [0, 0, 1, 0, 5, 5], core) == 1
    # entries outside [0, n)
    assert _forest_bad(dev, [0, -1, 1, 0, 2, 6], core) == 2
    # every point core (minPts <= 2): only the index order counts
    assert _forest_bad(dev, [0, 0, 1, 2, 2, 5], None) == 0
    assert _forest_bad(dev, [0, 2, 1, 2, 5, 5], None) == 2
    # a longer forest with planted violations at known places
    rng = np.random.default_rng(5)
    n = 100_000
    core = (rng.random(n) < 0.7).astype(np.uint8)
    cores = np.flatnonzero(core)
    parent = np.arange(n, dtype=np.int32)
    pos = np.arange(len(cores))
    earlier = cores[(rng.random(len(cores)) * pos).astype(np.int64)]   # a core before it (itself at 0)
    parent[cores] = np.where(rng.random(len(cores)) < 0.9, earlier, cores)
    non = np.flatnonzero(core == 0)
    claimed = non[rng.random(len(non)) < 0.5]
    parent[claimed] = cores[rng.integers(0, len(cores), size=len(claimed))]
    assert _forest_bad(dev, parent, core) == 0
    bad = parent.copy()
    plant = rng.choice(cores[(cores > 10) & (cores < n - 1)], size=37, replace=False)
    bad[plant] = np.minimum(plant + 1, n - 1)   # a core hooked under a larger index
    assert _forest_bad(dev, bad, core) == 37


@pytest.mark.parametrize("border", ["canonical", "first"])
@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_main_phase_leaves_a_valid_forest(dev, algo, border):
    import torch
    import paper_2103_05162_amd as fdb
    for name, scale in (("c1_blobs2d_16k", 1.0), ("c3_dense3d_8m", 1 / 64), ("c2_fof3d_2m", 1 / 16)):
        w = workload(name, scale)
        pts = torch.from_numpy(w.points).to(dev)
        h = fdb.Handle(0)
        _say(f"[gpu] forest check {algo}/{border} {w.name} n={w.n}")
        lab, core, k = fdb.dbscan(pts, w.eps, w.min_pts, algo=algo, border=border, handle=h, validate=True)
        assert h.last_info() & fdb.FDB_INFO_FOREST == 0, (name, algo, border)
        rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
        assert k == rk and np.array_equal(core.cpu().numpy(), rc)
        if border == "canonical":
            assert np.array_equal(lab.cpu().numpy(), rl)
        h.close()


def test_batched_main_phase_leaves_a_valid_forest(dev):
    import torch
    import paper_2103_05162_amd as fdb
    clouds, eps, mp = batched_clouds(num_clouds=48, lo=1024, hi=8192)
    offs = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(clouds)).to(dev)
    d_off, d_eps, d_mp = (torch.from_numpy(a).to(dev) for a in (offs, eps, mp))
    h = fdb.Handle(0)
    _say(f"[gpu] forest check batched: {len(clouds)} clouds")
    for border in ("canonical", "first"):
        lab, core, k = fdb.dbscan_batched(pts, d_off, d_eps, d_mp, algo="densebox", border=border, handle=h,
                                          validate=True)
        torch.cuda.synchronize()
        assert h.last_info() & fdb.FDB_INFO_FOREST == 0, border
        kk = k.cpu().numpy()
        for c in range(len(clouds)):
            assert kk[c] == oracle.dbscan(clouds[c], float(eps[c]), int(mp[c]))[2]
    h.close()
