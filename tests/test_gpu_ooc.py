"""Out-of-core batches: clouds held in host memory, clustered in groups of whole
clouds inside a device budget smaller than the batch needs. Every cloud's labels,
core flags and K must equal those of the in-core batched call (and so of the
cloud clustered alone)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


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


def _batch(seed, dim, num, empty_every=0):
    rng = np.random.default_rng(seed)
    clouds, eps, mp = [], [], []
    for c in range(num):
        n = 0 if empty_every and c % empty_every == 0 else int(np.exp(rng.uniform(np.log(50), np.log(6000))))
        k = int(rng.integers(1, 6))
        cen = rng.uniform(0, 1, size=(k, dim))
        lab = rng.integers(0, k, size=n)
        pts = cen[lab] + rng.uniform(0.003, 0.03) * rng.standard_normal((n, dim))
        noise = rng.random(n) < 0.2
        pts[noise] = rng.uniform(0, 1, size=(int(noise.sum()), dim))
        clouds.append(pts.astype(np.float32))
        eps.append(float(np.float32(rng.uniform(0.005, 0.04))))
        mp.append(int(rng.choice([1, 2, 3, 5, 10])))
    offs = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    allp = np.ascontiguousarray(np.concatenate(clouds)) if offs[-1] else np.zeros((0, dim), np.float32)
    return clouds, allp, offs, np.asarray(eps, np.float32), np.asarray(mp, np.int32)


def _in_core(dev, allp, offs, eps, mp, algo):
    import torch
    import paper_2103_05162_amd as fdb
    lab, core, k = fdb.dbscan_batched(torch.from_numpy(allp).to(dev), torch.from_numpy(offs).to(dev),
                                      torch.from_numpy(eps).to(dev), torch.from_numpy(mp).to(dev), algo=algo)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), core.cpu().numpy().astype(np.uint8), k.cpu().numpy()


def _budget_for(fdb, n_part, b_part, dim, algo):
    """A device budget whose slots hold about n_part points / b_part clouds."""
    return 2 * (fdb.workspace_bytes_batched(n_part, b_part, dim, algo) + n_part * (4 * dim + 5) + b_part * 24 + 4096)


@pytest.mark.parametrize("dim,algo", [(3, "densebox"), (2, "densebox"), (3, "fdbscan")])
def test_groups_equal_in_core_batch(dev, dim, algo):
    import torch
    import paper_2103_05162_amd as fdb
    clouds, allp, offs, eps, mp = _batch(40 + dim, dim, 300, empty_every=37)
    n, b = int(offs[-1]), len(clouds)
    budget = _budget_for(fdb, n // 5, b // 5, dim, algo)
    # the whole batch cannot be one group: it needs more than half the budget
    assert fdb.workspace_bytes_batched(n, b, dim, algo) > budget // 2
    _say(f"[gpu] out-of-core {algo} {dim}D: {b} clouds, {n} points, budget {budget >> 20} MiB")
    ref_l, ref_c, ref_k = _in_core(dev, allp, offs, eps, mp, algo)
    lab, core, k = fdb.dbscan_batched_host(allp, offs, eps, mp, budget, algo=algo)
    assert np.array_equal(k, ref_k)
    assert np.array_equal(lab, ref_l) and np.array_equal(core, ref_c)
    # pinned host buffers (copies overlap the clustering) give the same
    pin = torch.from_numpy(allp).pin_memory()
    lab_p = torch.empty(n, dtype=torch.int32).pin_memory()
    core_p = torch.empty(n, dtype=torch.uint8).pin_memory()
    lab2, core2, k2 = fdb.dbscan_batched_host(pin, offs, eps, mp, budget, algo=algo, labels=lab_p, is_core=core_p)
    assert np.array_equal(lab2, ref_l) and np.array_equal(core2, ref_c) and np.array_equal(k2, ref_k)
    assert np.array_equal(lab_p.numpy(), ref_l)
    # and a few clouds against the oracle itself
    for c in range(1, 300, 61):
        s, e = offs[c], offs[c + 1]
        ol, oc, ok = oracle.dbscan(clouds[c], float(eps[c]), int(mp[c]))
        assert k[c] == ok and np.array_equal(lab[s:e], ol) and np.array_equal(core[s:e].astype(bool), oc)


def test_nonfinite_cloud_isolated_and_nomem(dev):
    import paper_2103_05162_amd as fdb
    clouds, allp, offs, eps, mp = _batch(7, 3, 60)
    bad = 17
    allp = allp.copy()
    allp[offs[bad] + 1, 2] = np.inf
    budget = _budget_for(fdb, int(offs[-1]) // 4, 15, 3, "densebox")
    ref_l, ref_c, ref_k = _in_core(dev, allp, offs, eps, mp, "densebox")
    lab, core, k = fdb.dbscan_batched_host(allp, offs, eps, mp, budget)
    assert k[bad] == -1 and ref_k[bad] == -1
    good = np.ones(len(clouds), bool)
    good[bad] = False
    assert np.array_equal(k[good], ref_k[good])
    keep = np.ones(int(offs[-1]), bool)
    keep[offs[bad]:offs[bad + 1]] = False
    assert np.array_equal(lab[keep], ref_l[keep]) and np.array_equal(core[keep], ref_c[keep])
    # a budget too small for the largest cloud is refused before any work
    big = int(np.argmax(np.diff(offs)))
    small = _budget_for(fdb, int(offs[big + 1] - offs[big]) // 2, 1, 3, "densebox")
    with pytest.raises(fdb.FdbError) as e:
        fdb.dbscan_batched_host(allp, offs, eps, mp, small)
    assert e.value.status == 2
    # offsets must start at 0 and not decrease
    bad_offs = offs.copy()
    bad_offs[5], bad_offs[6] = bad_offs[6], bad_offs[5]
    if bad_offs[5] != bad_offs[6]:
        with pytest.raises(fdb.FdbError) as e:
            fdb.dbscan_batched_host(allp, bad_offs, eps, mp, budget)
        assert e.value.status == 1


def test_groups_of_mixed_shapes(dev):
    """Many tiny clouds around two large ones in a budget that holds one large
    cloud per slot: groups of very different point and cloud counts share the
    slots (each group is laid out on its own), results equal the in-core batch."""
    import paper_2103_05162_amd as fdb
    for dim in (3, 2):
        rng = np.random.default_rng(60 + dim)
        sizes = [int(x) for x in rng.integers(5, 60, size=300)]
        sizes[120] = sizes[240] = 40000
        clouds = []
        for n in sizes:
            cen = rng.uniform(0, 1, size=(3, dim))
            pts = cen[rng.integers(0, 3, size=n)] + 0.01 * rng.standard_normal((n, dim))
            clouds.append(pts.astype(np.float32))
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        allp = np.ascontiguousarray(np.concatenate(clouds))
        eps = np.full(len(sizes), 0.01, np.float32)
        mp = np.full(len(sizes), 4, np.int32)
        budget = _budget_for(fdb, 40000, 1, dim, "densebox") + (1 << 20)
        _say(f"[gpu] out-of-core mixed groups {dim}D: {len(sizes)} clouds, budget {budget >> 20} MiB")
        ref_l, ref_c, ref_k = _in_core(dev, allp, offs, eps, mp, "densebox")
        lab, core, k = fdb.dbscan_batched_host(allp, offs, eps, mp, budget)
        assert np.array_equal(k, ref_k) and np.array_equal(lab, ref_l) and np.array_equal(core, ref_c)
