"""Served clustering: jobs submitted to a server (continuous batching under an
HBM budget, or one at a time) must give each job exactly the labels, core flags
and K it gets alone, whatever it was batched with."""
import sys

import numpy as np
import pytest

import oracle
from workloads.gen import mixture_cloud

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


def _jobs(seed, count, lo=200, hi=20000):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.choice([2, 3]))
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        pts = mixture_cloud(rng, n, d=d)
        out.append((pts, float(np.float32(rng.uniform(0.005, 0.03))), int(rng.choice([1, 2, 5, 10]))))
    return out


def _upload(dev, jobs):
    """Device copies of the jobs' points, and their output buffers (synchronised)."""
    import torch
    bufs = []
    for pts, eps, mp in jobs:
        t = torch.from_numpy(pts).to(dev)
        lab = torch.full((len(pts),), -7, dtype=torch.int32, device=dev)
        core = torch.zeros(len(pts), dtype=torch.uint8, device=dev)
        bufs.append((t, lab, core))
    torch.cuda.synchronize()
    return bufs


def _submit_all(srv, dev, jobs):
    bufs = _upload(dev, jobs)
    tickets = [srv.submit_raw(t.data_ptr(), t.shape[0], t.shape[1], eps, mp, lab.data_ptr(), core.data_ptr())
               for (t, lab, core), (_, eps, mp) in zip(bufs, jobs)]
    return bufs, tickets


def _alone(dev, pts, eps, mp, algo):
    import torch
    import paper_2103_05162_amd as fdb
    lab, core, k = fdb.dbscan(torch.from_numpy(pts).to(dev), eps, mp, algo=algo)
    return lab.cpu().numpy(), core.cpu().numpy(), k


@pytest.mark.parametrize("algo", ["fdbscan", "densebox"])
def test_served_batches_equal_jobs_alone(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    jobs = _jobs(11, 48)
    # a large first job keeps the device busy while the others queue up behind it
    rng = np.random.default_rng(12)
    jobs.insert(0, (rng.uniform(0, 1, size=(3_000_000, 3)).astype(np.float32), 0.004, 5))
    _say(f"[gpu] serve {len(jobs)} jobs ({algo}), {sum(len(j[0]) for j in jobs)} points")
    srv = fdb.Server(0, budget_bytes=4 << 30, max_batch=64, mode="batched", algo=algo)
    try:
        bufs, tickets = _submit_all(srv, dev, jobs)
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    _say(f"[gpu] batches {st['batches']}, largest {st['max_batch_jobs']} jobs, p99 {st['p99_us']:.0f} us")
    assert st["jobs"] == len(jobs) and st["max_batch_jobs"] >= 2
    for (pts, eps, mp), (t, lab, core), r in zip(jobs, bufs, res):
        assert r["done"] and r["status"] == 0
        rl, rc, rk = _alone(dev, pts, eps, mp, algo)
        assert r["num_clusters"] == rk
        assert np.array_equal(lab.cpu().numpy(), rl) and np.array_equal(core.cpu().numpy(), rc)
    # and the small ones against the oracle itself
    for (pts, eps, mp), (t, lab, core) in list(zip(jobs, bufs))[1:9]:
        ol, oc, ok = oracle.dbscan(pts, eps, mp)
        assert np.array_equal(lab.cpu().numpy(), ol)


def test_budget_admission_and_fifo(dev):
    import torch
    import paper_2103_05162_amd as fdb
    jobs = _jobs(13, 24, lo=1000, hi=60000)
    budget = 24 << 20  # two slots of 12 MiB in batched mode
    srv = fdb.Server(0, budget_bytes=budget, max_batch=1024, mode="batched")
    fifo = fdb.Server(0, budget_bytes=budget, mode="fifo")
    try:
        # a job that alone exceeds the budget is refused at submission
        big = torch.zeros((1_000_000, 3), dtype=torch.float32, device=dev)
        lab = torch.empty(1_000_000, dtype=torch.int32, device=dev)
        with pytest.raises(fdb.FdbError) as e:
            srv.submit_raw(big.data_ptr(), big.shape[0], 3, 0.01, 5, lab.data_ptr())
        assert e.value.status == 2
        with pytest.raises(fdb.FdbError) as e:
            srv.submit_raw(big.data_ptr(), big.shape[0], 3, 0.0, 5, lab.data_ptr())
        assert e.value.status == 1
        bufs, tickets = _submit_all(srv, dev, jobs)
        bufs2, tickets2 = _submit_all(fifo, dev, jobs)
        srv.drain()
        fifo.drain()
        st, st2 = srv.stats(), fifo.stats()
        assert st["jobs"] == len(jobs) and st2["jobs"] == len(jobs)
        assert st2["max_batch_jobs"] == 1 and st2["batches"] == len(jobs)
        assert st["batches"] >= 2  # the budget splits the queue into several launches
        for (pts, eps, mp), (t, l1, c1), (t2, l2, c2), a, b in zip(jobs, bufs, bufs2, tickets, tickets2):
            r1, r2 = srv.poll(a), fifo.poll(b)
            assert r1["status"] == 0 and r2["status"] == 0 and r1["num_clusters"] == r2["num_clusters"]
            assert torch.equal(l1, l2) and torch.equal(c1, c2)
        for (pts, eps, mp), (t, l1, c1) in [jb for jb in zip(jobs, bufs) if len(jb[0][0]) <= 20000][:6]:
            ol, oc, ok = oracle.dbscan(pts, eps, mp)
            assert np.array_equal(l1.cpu().numpy(), ol) and np.array_equal(c1.cpu().numpy().astype(bool), oc)
    finally:
        srv.close()
        fifo.close()


def test_nonfinite_job_is_isolated_and_empty_job(dev):
    import torch
    import paper_2103_05162_amd as fdb
    jobs = _jobs(14, 6, lo=500, hi=3000)
    bad = jobs[2][0].copy()
    bad[5, 0] = np.nan
    jobs[2] = (bad, jobs[2][1], jobs[2][2])
    jobs = [j for j in jobs if j[0].shape[1] == 3] + [j for j in jobs if j[0].shape[1] == 2]
    srv = fdb.Server(0, budget_bytes=1 << 30, max_batch=64)
    try:
        bufs, tickets = _submit_all(srv, dev, jobs)
        lab0 = torch.empty(0, dtype=torch.int32, device=dev)
        t0 = srv.submit_raw(0, 0, 3, 0.1, 3, 0)
        srv.drain()
        assert srv.poll(t0)["done"] and srv.poll(t0)["num_clusters"] == 0
        del lab0
        for (pts, eps, mp), (t, lab, core), tk in zip(jobs, bufs, tickets):
            r = srv.poll(tk)
            if np.isfinite(pts).all():
                assert r["status"] == 0
                ol, oc, ok = oracle.dbscan(pts, eps, mp)
                assert r["num_clusters"] == ok and np.array_equal(lab.cpu().numpy(), ol)
            else:
                assert r["status"] == 4 and r["num_clusters"] == -1
    finally:
        srv.close()


def test_small_job_is_launched_while_a_large_one_runs(dev):
    """Two slots: a small job submitted while a large job's batch is on the device is
    launched at once in the other slot, before the large job is done, instead of
    waiting for it (whether the device then runs the two batches side by side is up
    to its queues); each job's labels, core flags and K are those it gets alone."""
    import time
    import torch
    import paper_2103_05162_amd as fdb
    rng = np.random.default_rng(21)
    big = (mixture_cloud(rng, 2_000_000, d=3), 0.02, 5)
    small = (mixture_cloud(rng, 4000, d=3), 0.02, 5)
    srv = fdb.Server(0, budget_bytes=8 << 30, max_batch=64, mode="batched", algo="densebox")
    try:
        (bt, bl, bc), (st_, sl_, sc_) = _upload(dev, [big, small])
        _say(f"[gpu] two slots: big job n={bt.shape[0]}, small job n={st_.shape[0]}")
        tb = srv.submit_raw(bt.data_ptr(), bt.shape[0], 3, big[1], big[2], bl.data_ptr(), bc.data_ptr())
        t0 = time.perf_counter()
        while srv.poll(tb)["queue_us"] < 0:  # until the big job's batch is taken
            if time.perf_counter() - t0 > 10:
                raise AssertionError("the big job was not launched")
        ts = srv.submit_raw(st_.data_ptr(), st_.shape[0], 3, small[1], small[2], sl_.data_ptr(), sc_.data_ptr())
        delta_us = (time.perf_counter() - t0) * 1e6  # bounds the gap between the two submissions
        srv.drain()
        rb, rs = srv.poll(tb), srv.poll(ts)
        assert rb["status"] == 0 and rs["status"] == 0
        assert rb["batch_jobs"] == 1 and rs["batch_jobs"] == 1, "the jobs were batched together"
        assert srv.stats()["batches"] == 2
        # the small job's batch started before the big job was done
        assert rs["queue_us"] + delta_us < rb["latency_us"], (rs, rb, delta_us)
        _say(f"[gpu] big job {rb['latency_us']:.0f} us, small job {rs['latency_us']:.0f} us "
             f"(queued {rs['queue_us']:.0f} us), submitted {delta_us:.0f} us apart")
        for (pts, eps, mp), lab, core, r in ((big, bl, bc, rb), (small, sl_, sc_, rs)):
            al, ac, ak = _alone(dev, pts, eps, mp, "densebox")
            assert r["num_clusters"] == ak
            assert np.array_equal(lab.cpu().numpy(), al) and np.array_equal(core.cpu().numpy().astype(bool), ac)
        ol, oc, ok = oracle.dbscan(small[0], small[1], small[2])
        assert rs["num_clusters"] == ok and np.array_equal(sl_.cpu().numpy(), ol)
    finally:
        srv.close()
