"""The boundary's asynchronous contract and the launch-shape machinery, through
the C ABI on one GPU:

* fdb_dbscan with DenseBox waits for nothing when no K is asked for, so a
  stream capture records the whole call into a HIP graph; every replay (with
  eager work and synchronisations between replays) equals the eager call and
  the oracle;
* FDB_FLAG_GRAPH (the library's own recorded launch sequences) for single and
  batched calls;
* a caller workspace one byte short is refused before any launch;
* fdb_last_status reports device-side errors of an asynchronous call;
* the autotuner's table: persisted, read back by a new handle, and the tuned
  shape gives the oracle's labels.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads.gen import workload

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


def _bufs(dev, n, d, algo):
    import torch
    import paper_2103_05162_amd as fdb
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(fdb.workspace_bytes(n, d, algo), dtype=torch.uint8, device=dev)
    return labels, core, ws


@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_stream_capture_of_one_call_replays_exactly(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    w = workload("c3_dense3d_8m", 1 / 64)
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    pts = torch.from_numpy(w.points).to(dev)
    labels, core, ws = _bufs(dev, w.n, 3, algo)
    h = fdb.Handle(0)
    kw = dict(algo=algo, handle=h, labels=labels, is_core=core, workspace=ws, want_k=False)
    _say(f"[gpu] stream capture {algo} n={w.n}")
    fdb.dbscan(pts, w.eps, w.min_pts, **kw)           # eager
    torch.cuda.synchronize()
    eager = (labels.cpu().numpy().copy(), core.cpu().numpy().copy())
    assert np.array_equal(eager[0], rl) and np.array_equal(eager[1], rc)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            fdb.dbscan(pts, w.eps, w.min_pts, **kw)
    torch.cuda.synchronize()
    for r in range(4):
        labels.fill_(-7)
        core.fill_(9)
        g.replay()
        torch.cuda.synchronize()
        got_l, got_c = labels.cpu().numpy(), core.cpu().numpy()
        assert np.array_equal(got_l, rl), f"replay {r}: labels"
        assert np.array_equal(got_c, rc), f"replay {r}: core flags"
        # eager work between replays on the same buffers
        fdb.dbscan(pts, w.eps, w.min_pts, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(labels.cpu().numpy(), rl)
    st, info = h.last_status(torch.cuda.current_stream().cuda_stream)
    assert st == 0 and info == 0
    h.close()


@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_library_graph_flag_single_call(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    w = workload("c2_fof3d_2m", 1 / 32)
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    pts = torch.from_numpy(w.points).to(dev)
    labels, core, ws = _bufs(dev, w.n, 3, algo)
    h = fdb.Handle(0)
    _say(f"[gpu] FDB_FLAG_GRAPH single {algo} n={w.n}")
    for r in range(5):
        labels.fill_(-7)
        _, _, k = fdb.dbscan(pts, w.eps, w.min_pts, algo=algo, handle=h, labels=labels, is_core=core, workspace=ws,
                             graph=True, want_k=(r % 2 == 0))
        torch.cuda.synchronize()
        if k is not None:
            assert k == rk
        assert np.array_equal(labels.cpu().numpy(), rl), f"call {r}"
        assert np.array_equal(core.cpu().numpy().astype(bool), rc), f"call {r}"
    h.close()


def test_library_graph_flag_batched(dev):
    import torch
    import paper_2103_05162_amd as fdb
    from workloads.gen import batched_clouds
    clouds, eps, mp = batched_clouds(num_clouds=64, lo=1024, hi=8192)
    sizes = [len(c) for c in clouds]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(clouds)).to(dev)
    n = int(offs[-1])
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    k = torch.empty(len(clouds), dtype=torch.int32, device=dev)
    d_off, d_eps, d_mp = (torch.from_numpy(a).to(dev) for a in (offs, eps, mp))
    ws = torch.empty(fdb.workspace_bytes_batched(n, len(clouds), 3, "densebox"), dtype=torch.uint8, device=dev)
    refs = [oracle.dbscan(c, float(eps[i]), int(mp[i])) for i, c in enumerate(clouds)]
    h = fdb.Handle(0)
    _say(f"[gpu] FDB_FLAG_GRAPH batched: {len(clouds)} clouds, {n} points")
    for r in range(4):
        labels.fill_(-7)
        fdb.dbscan_batched(pts, d_off, d_eps, d_mp, algo="densebox", handle=h, labels=labels, is_core=core,
                           num_clusters=k, workspace=ws, graph=True)
        torch.cuda.synchronize()
        lab, co, kk = labels.cpu().numpy(), core.cpu().numpy().astype(bool), k.cpu().numpy()
        for c, (rl, rc, rk) in enumerate(refs):
            sl = slice(offs[c], offs[c + 1])
            assert kk[c] == rk and np.array_equal(lab[sl], rl) and np.array_equal(co[sl], rc), (r, c)
        assert h.last_info() == 0
    h.close()


@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_caller_workspace_one_byte_short_is_refused(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    w = workload("c1_blobs2d_16k")
    pts = torch.from_numpy(w.points).to(dev)
    need = fdb.workspace_bytes(w.n, 2, algo)
    labels = torch.full((w.n,), -7, dtype=torch.int32, device=dev)
    short = torch.empty(need - 1, dtype=torch.uint8, device=dev)
    with pytest.raises(fdb.FdbError) as e:
        fdb.dbscan(pts, w.eps, w.min_pts, algo=algo, labels=labels, workspace=short)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert (labels == -7).all().item(), "outputs touched by a refused call"
    exact = torch.empty(need, dtype=torch.uint8, device=dev)
    lab, core, k = fdb.dbscan(pts, w.eps, w.min_pts, algo=algo, workspace=exact)
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    assert k == rk and np.array_equal(lab.cpu().numpy(), rl)


@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_last_status_reports_device_errors_of_an_async_call(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    rng = np.random.default_rng(13)
    pts = rng.uniform(0, 1, size=(5000, 3)).astype(np.float32)
    pts[123, 0] = np.inf
    t = torch.from_numpy(pts).to(dev)
    h = fdb.Handle(0)
    fdb.dbscan(t, 0.05, 4, algo=algo, handle=h, want_k=False)
    st, info = h.last_status(torch.cuda.current_stream().cuda_stream)
    assert st == 4 and info & fdb.FDB_INFO_NONFINITE
    good = torch.from_numpy(rng.uniform(0, 1, size=(5000, 3)).astype(np.float32)).to(dev)
    fdb.dbscan(good, 0.05, 4, algo=algo, handle=h, want_k=False)
    st, info = h.last_status(torch.cuda.current_stream().cuda_stream)
    assert st == 0 and info == 0
    h.close()


def test_tuner_table_is_persisted_and_used(dev, tmp_path, monkeypatch):
    import torch
    import paper_2103_05162_amd as fdb
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FDB_TUNE_CACHE", str(cache))
    w = workload("c3_dense3d_8m", 1 / 32)
    pts = torch.from_numpy(w.points).to(dev)
    h = fdb.Handle(0)
    _say(f"[gpu] tuning densebox n={w.n}")
    best, ms, ms0 = fdb.tune(pts, w.eps, w.min_pts, algo="densebox", reps=2, handle=h)
    assert ms <= ms0 + 1e-9 and best["leaf_size"] in (4, 8, 16, 32) and best["block_size"] in (64, 128, 256)
    assert best["tile"] in (32, 64)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fdbtune1 0 1 3 ")
    tuned = fdb.options_dict(h.tuned_options(w.n, 3, w.min_pts, 0, fdb.make_options("densebox")))
    assert (tuned["leaf_size"], tuned["block_size"], tuned["tile"]) == \
        (best["leaf_size"], best["block_size"], best["tile"])
    h.close()
    h2 = fdb.Handle(0)  # reads the cache file back
    again = fdb.options_dict(h2.tuned_options(w.n, 3, w.min_pts, 0, fdb.make_options("densebox")))
    assert again == tuned
    # another class (minPts <= 2) keeps the defaults
    other = fdb.options_dict(h2.tuned_options(w.n, 3, 2, 0, fdb.make_options("densebox")))
    assert (other["leaf_size"], other["block_size"], other["tile"]) == (8, 128, 64)
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    lab, core, k = fdb.dbscan(pts, w.eps, w.min_pts, algo="densebox", handle=h2)  # tuned shape
    assert k == rk and np.array_equal(lab.cpu().numpy(), rl) and np.array_equal(core.cpu().numpy(), rc)
    for leaf, block, tile in ((4, 64, 32), (32, 256, 8)):
        lab, core, k = fdb.dbscan(pts, w.eps, w.min_pts, algo="densebox", handle=h2, leaf_size=leaf,
                                  block_size=block, tile=tile)
        assert k == rk and np.array_equal(lab.cpu().numpy(), rl), (leaf, block, tile)
    h2.close()
