"""fdb_dbscan_noalloc through the C ABI on one GPU: the allocation-free variant of
fdb_dbscan, working in the library's static device scratch, gives exactly what
fdb_dbscan gives (labels, core flags, K) on two calls in a row, the second with a
smaller input (the scratch keeps the first call's contents); an input too large
for the scratch and a graph request are refused before any launch.
"""
import sys

import numpy as np
import pytest

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


def _plain(fdb, h, pts, eps, mp, algo, border):
    lab, core, k = fdb.dbscan(pts, eps, mp, algo=algo, border=border, handle=h)
    return lab.cpu().numpy(), core.cpu().numpy(), k


@pytest.mark.parametrize("border", ["canonical", "none"])
@pytest.mark.parametrize("algo", ["densebox", "fdbscan"])
def test_noalloc_equals_fdb_dbscan_on_two_calls(dev, algo, border):
    import torch
    import paper_2103_05162_amd as fdb
    big = workload("c3_dense3d_8m", 1 / 32)     # 262,144 3D points: about 58 MiB of DenseBox workspace
    small = workload("c1_blobs2d_16k")          # then a smaller 2D input in the same scratch
    assert fdb.workspace_bytes(big.n, 3, algo) <= fdb.FDB_NOALLOC_SCRATCH_BYTES
    h_plain = fdb.Handle(0)
    h = fdb.Handle(0)
    for w in (big, small):
        pts = torch.from_numpy(w.points).to(dev)
        d = w.points.shape[1]
        _say(f"[gpu] noalloc {algo}/{border} {w.name} n={w.n} d={d}")
        rl, rc, rk = _plain(fdb, h_plain, pts, w.eps, w.min_pts, algo, border)
        labels = torch.full((w.n,), -7, dtype=torch.int32, device=dev)
        core = torch.full((w.n,), 9, dtype=torch.uint8, device=dev)
        k = fdb.dbscan_noalloc(pts, w.eps, w.min_pts, labels, core, algo=algo, border=border, handle=h)
        torch.cuda.synchronize()
        assert k == rk, (w.name, k, rk)
        assert np.array_equal(labels.cpu().numpy(), rl), w.name
        assert np.array_equal(core.cpu().numpy(), rc.view(np.uint8)), w.name
    h.close()
    h_plain.close()


def test_noalloc_asynchronous_call_then_status(dev):
    import torch
    import paper_2103_05162_amd as fdb
    w = workload("c2_fof3d_2m", 1 / 16)  # 131,072 points, minPts 2
    pts = torch.from_numpy(w.points).to(dev)
    rl, rc, rk = _plain(fdb, fdb.Handle(0), pts, w.eps, w.min_pts, "densebox", "canonical")
    labels = torch.empty(w.n, dtype=torch.int32, device=dev)
    core = torch.empty(w.n, dtype=torch.uint8, device=dev)
    h = fdb.Handle(0)
    _say(f"[gpu] noalloc without K, n={w.n}")
    assert fdb.dbscan_noalloc(pts, w.eps, w.min_pts, labels, core, algo="densebox", handle=h, want_k=False) is None
    st, info = h.last_status(torch.cuda.current_stream().cuda_stream)
    assert st == 0 and info == 0
    assert np.array_equal(labels.cpu().numpy(), rl)
    h.close()


def test_noalloc_refuses_what_the_scratch_cannot_hold(dev):
    import torch
    import paper_2103_05162_amd as fdb
    h = fdb.Handle(0)
    n = 1
    while fdb.workspace_bytes(n, 3, "densebox") <= fdb.FDB_NOALLOC_SCRATCH_BYTES:
        n *= 2
    pts = torch.zeros((n, 3), dtype=torch.float32, device=dev)
    labels = torch.full((n,), -7, dtype=torch.int32, device=dev)
    core = torch.full((n,), 9, dtype=torch.uint8, device=dev)
    _say(f"[gpu] noalloc refusal n={n}")
    with pytest.raises(fdb.FdbError) as e:
        fdb.dbscan_noalloc(pts, 0.1, 5, labels, core, algo="densebox", handle=h)
    assert e.value.status == fdb.FDB_ERR_SCRATCH
    small = pts[:1000]
    with pytest.raises(fdb.FdbError) as e:  # a graph recording would allocate
        lib = fdb.load()
        opt = fdb.make_options("densebox", graph=True)
        h.dbscan_noalloc_raw(small.data_ptr(), 1000, 3, 0.1, 5, labels.data_ptr(), core.data_ptr(),
                             torch.cuda.current_stream().cuda_stream, opt)
    assert e.value.status == 1
    torch.cuda.synchronize()
    assert (labels == -7).all().item() and (core == 9).all().item(), "outputs touched by a refused call"
    h.close()
