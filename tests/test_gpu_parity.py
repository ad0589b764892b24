"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Canonical mode must match the oracle bit for bit (labels, core flags, K) for
both algorithms; first-claim mode (the paper's border rule) must match up to
the free choice of a border point's cluster. Sizes span many sort tiles,
traversal workgroups and a ragged tail; edge cases cover the degenerate inputs
the method has.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import assert_tolerance_mode
from workloads.gen import workload

pytestmark = pytest.mark.gpu

ALGOS = ["fdbscan", "densebox"]


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


def run_gpu(dev, pts, eps, min_pts, algo="fdbscan", border="canonical", **kw):
    import torch
    import paper_2103_05162_amd as fdb
    t = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).to(dev)
    labels, core, k = fdb.dbscan(t, eps, min_pts, algo=algo, border=border, **kw)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), core.cpu().numpy(), k


def assert_exact(dev, pts, eps, min_pts, algo, ref=None, **kw):
    _say(f"[gpu] n={len(pts)} d={pts.shape[1]} eps={eps} minPts={min_pts} algo={algo} {kw}")
    if ref is None:
        ref = oracle.dbscan(pts, eps, min_pts)
    lab, core, k = run_gpu(dev, pts, eps, min_pts, algo, **kw)
    rl, rc, rk = ref
    assert k == rk, f"K {k} != {rk}"
    assert np.array_equal(core, rc), f"core differs at {np.flatnonzero(core != rc)[:10]}"
    bad = np.flatnonzero(lab != rl)
    assert bad.size == 0, f"{bad.size} labels differ, first {bad[:10]}: gpu {lab[bad[:10]]} ref {rl[bad[:10]]}"
    return ref


# ---- the configured workloads (full C1; reduced C2/C3 with their density) ------

@pytest.mark.parametrize("algo", ALGOS)
def test_c1_full_canonical(dev, algo):
    w = workload("c1_blobs2d_16k")
    assert_exact(dev, w.points, w.eps, w.min_pts, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_c1_first_claim_mode(dev, algo):
    w = workload("c1_blobs2d_16k")
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    _say(f"[gpu] c1 first-claim {algo}")
    lab, core, k = run_gpu(dev, w.points, w.eps, w.min_pts, algo, border="first")
    assert k == rk
    assert_tolerance_mode(w.points, w.eps, lab, core, rl, rc, oracle.check_border)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("scale", [1 / 16])
def test_c2_reduced_canonical(dev, algo, scale):
    w = workload("c2_fof3d_2m", scale)
    assert_exact(dev, w.points, w.eps, w.min_pts, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_c3_reduced_canonical(dev, algo):
    w = workload("c3_dense3d_8m", 1 / 64)
    assert_exact(dev, w.points, w.eps, w.min_pts, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_c3_reduced_first_claim_mode(dev, algo):
    w = workload("c3_dense3d_8m", 1 / 64)
    rl, rc, rk = oracle.dbscan(w.points, w.eps, w.min_pts)
    _say(f"[gpu] c3/64 first-claim {algo}")
    lab, core, k = run_gpu(dev, w.points, w.eps, w.min_pts, algo, border="first")
    assert k == rk
    assert_tolerance_mode(w.points, w.eps, lab, core, rl, rc, oracle.check_border)


# ---- both algorithms, border-rich mixtures, several parameter choices -----------

def _mixture(seed, n, d, k, sigma, noise=0.3):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, size=(k, d))
    lab = rng.integers(0, k, size=n)
    pts = c[lab] + sigma * rng.standard_normal((n, d))
    m = rng.random(n) < noise
    pts[m] = rng.uniform(0, 1, size=(int(m.sum()), d))
    return pts.astype(np.float32)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("d,n,eps,mp,seed", [
    (2, 30011, 0.004, 5, 1), (3, 40009, 0.02, 10, 2), (3, 20011, 0.03, 3, 3), (2, 25013, 0.006, 2, 4),
    (3, 12007, 0.015, 1, 5), (2, 9001, 0.01, 30, 6),
])
def test_mixtures_canonical(dev, algo, d, n, eps, mp, seed):
    pts = _mixture(seed, n, d, 12, 0.01)
    assert_exact(dev, pts, eps, mp, algo)


@pytest.mark.parametrize("leaf,block", [(1, 64), (2, 128), (8, 256), (16, 512), (32, 1024)])
def test_leaf_and_block_sizes_do_not_change_labels(dev, leaf, block):
    pts = _mixture(7, 20000, 3, 10, 0.01)
    ref = oracle.dbscan(pts, 0.02, 6)
    for algo in ALGOS:
        assert_exact(dev, pts, 0.02, 6, algo, ref=ref, leaf_size=leaf, block_size=block)


# ---- edge cases ----------------------------------------------------------------------

@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 4095, 4096, 4097, 5631, 5632, 5633, 6143, 6144, 6145, 8193,
                               11265, 12289])
def test_ragged_sizes(dev, algo, n):
    # sort tiles: 5632 32-bit keys (grid keys), 6144 64-bit keys (Morton codes)
    pts = _mixture(100 + n, n, 3, 3, 0.02)
    for mp in (1, 2, 4):
        assert_exact(dev, pts, 0.05, mp, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_empty_input(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    t = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    lab, core, k = fdb.dbscan(t, 0.1, 3, algo=algo)
    assert k == 0 and lab.numel() == 0


@pytest.mark.parametrize("algo", ALGOS)
def test_all_duplicates(dev, algo):
    pts = np.full((5000, 3), 0.25, np.float32)
    assert_exact(dev, pts, 1e-4, 10, algo)
    assert_exact(dev, pts, 1e-4, 5000, algo)
    assert_exact(dev, pts, 1e-4, 5001, algo)
    assert_exact(dev, pts, 1e-4, 2, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_degenerate_extent_and_exact_distances(dev, algo):
    # points on a line (zero extent on two axes) with dyadic spacing = eps
    x = np.arange(3000, dtype=np.float32) * np.float32(0.125)
    pts = np.stack([x, np.zeros_like(x), np.zeros_like(x)], 1)
    pts[::7, 0] += np.float32(0.0625)
    assert_exact(dev, pts, 0.125, 3, algo)
    # 2D unit lattice, eps = 1 exactly: interior points have 5 neighbours
    g = np.stack(np.meshgrid(np.arange(120), np.arange(90), indexing="ij"), -1).reshape(-1, 2).astype(np.float32)
    assert_exact(dev, g, 1.0, 5, algo)
    assert_exact(dev, g, 1.0, 6, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_eps_extremes(dev, algo):
    pts = _mixture(9, 6000, 2, 4, 0.02)
    assert_exact(dev, pts, 10.0, 7, algo)       # one cluster
    assert_exact(dev, pts, 1e-7, 2, algo)       # all noise
    assert_exact(dev, pts, 1e-7, 1, algo)       # every point its own cluster


def test_densebox_falls_back_when_the_grid_cannot_be_keyed(dev):
    import paper_2103_05162_amd as fdb
    rng = np.random.default_rng(3)
    pts = (rng.uniform(0, 1e7, size=(3000, 2))).astype(np.float32)
    pts[:100] = pts[0] + rng.uniform(0, 1e-3, size=(100, 2)).astype(np.float32)
    ref = oracle.dbscan(pts, 2e-3, 5)
    assert_exact(dev, pts, 2e-3, 5, "densebox", ref=ref)
    assert fdb.default_handle(0).last_info() & fdb.FDB_INFO_DENSEBOX_FALLBACK
    assert_exact(dev, pts, 2e-3, 5, "fdbscan", ref=ref)
    assert not fdb.default_handle(0).last_info() & fdb.FDB_INFO_DENSEBOX_FALLBACK


@pytest.mark.parametrize("algo", ALGOS)
def test_nonfinite_input_is_reported(dev, algo):
    import torch
    import paper_2103_05162_amd as fdb
    pts = _mixture(11, 1000, 3, 2, 0.02)
    pts[17, 1] = np.nan
    t = torch.from_numpy(pts).to(dev)
    with pytest.raises(fdb.FdbError) as e:
        fdb.dbscan(t, 0.05, 4, algo=algo)
    assert e.value.status == 4


def test_invalid_arguments_are_rejected(dev):
    import torch
    import paper_2103_05162_amd as fdb
    t = torch.zeros((10, 3), dtype=torch.float32, device=dev)
    for eps, mp in ((0.0, 3), (-1.0, 3), (float("nan"), 3), (float("inf"), 3), (0.1, 0)):
        with pytest.raises(fdb.FdbError) as e:
            fdb.dbscan(t, eps, mp)
        assert e.value.status == 1


# ---- metamorphic and repeatability ----------------------------------------------

@pytest.mark.parametrize("algo", ALGOS)
def test_reflection_and_scaling_give_identical_labels(dev, algo):
    pts = _mixture(12, 30000, 3, 8, 0.01)
    eps, mp = 0.015, 5
    base = run_gpu(dev, pts, eps, mp, algo)
    for q, e in ((-pts, eps), (pts[:, [1, 0, 2]].copy(), eps), (pts * np.float32(64.0), eps * 64.0)):
        got = run_gpu(dev, np.ascontiguousarray(q), e, mp, algo)
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])


@pytest.mark.parametrize("algo", ALGOS)
def test_repeated_runs_are_identical(dev, algo):
    w = workload("c3_dense3d_8m", 1 / 128)
    first = run_gpu(dev, w.points, w.eps, w.min_pts, algo)
    for _ in range(5):
        again = run_gpu(dev, w.points, w.eps, w.min_pts, algo)
        assert np.array_equal(again[0], first[0]) and np.array_equal(again[1], first[1])


def test_fdbscan_and_densebox_agree(dev):
    pts = _mixture(13, 50000, 3, 20, 0.004, noise=0.2)
    a = run_gpu(dev, pts, 0.01, 8, "fdbscan")
    b = run_gpu(dev, pts, 0.01, 8, "densebox")
    assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("d", [2, 3])
def test_border_records_overflow_and_walk_fallback(dev, algo, d):
    """Most points non-core with one neighbour (pairs): more border records than
    the record buffer holds (n/8), so the rest take the walk path; plus blobs
    whose fringe points have more neighbours than a record keeps (minPts 12)."""
    rng = np.random.default_rng(40 + d)
    eps = 0.01
    npairs = 30000
    side = int(np.ceil(npairs ** (1 / d)))
    grid = np.stack(np.meshgrid(*[np.arange(side)] * d, indexing="ij"), -1).reshape(-1, d)[:npairs]
    a = grid * (4 * eps) + rng.uniform(0, eps, size=(npairs, d))
    off = rng.standard_normal((npairs, d))
    off *= (0.5 * eps) / np.linalg.norm(off, axis=1, keepdims=True)
    pairs = np.concatenate([a, a + off])
    blobs = [rng.uniform(0, side * 4 * eps, size=d) + 0.6 * eps * rng.standard_normal((400, d)) for _ in range(12)]
    pts = np.concatenate([pairs] + blobs).astype(np.float32)
    pts = pts[rng.permutation(len(pts))]
    for mp in (3, 12):
        assert_exact(dev, pts, eps, mp, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_unaligned_input_pointer(dev, algo):
    """Points starting 12 bytes into an allocation (not 16-byte aligned) take the
    scalar bounds path; labels must not change."""
    import torch
    import paper_2103_05162_amd as fdb
    pts = _mixture(77, 20001, 3, 12, 0.01)
    base = torch.from_numpy(np.concatenate([np.zeros((1, 3), np.float32), pts])).to(dev)
    view = base[1:]
    assert view.data_ptr() % 16 != 0
    ref = oracle.dbscan(pts, 0.01, 5)
    lab, core, k = fdb.dbscan(view, 0.01, 5, algo=algo)
    torch.cuda.synchronize()
    assert k == ref[2]
    assert np.array_equal(lab.cpu().numpy(), ref[0]) and np.array_equal(core.cpu().numpy(), ref[1])


_MANY_CELLS = {}


def _many_cells_case():
    if not _MANY_CELLS:
        rng = np.random.default_rng(91)
        k, per = 700_000, 6
        centers = rng.uniform(0, 1, size=(k, 3))
        pts = (np.repeat(centers, per, axis=0) + 1e-4 * rng.standard_normal((k * per, 3))).astype(np.float32)
        pts = pts[rng.permutation(len(pts))]
        eps, mp = 0.003, 4
        _MANY_CELLS["case"] = (pts, eps, mp, oracle.dbscan(pts, eps, mp))
    return _MANY_CELLS["case"]


@pytest.mark.parametrize("border", ["canonical", "first"])
def test_many_dense_cells(dev, border):
    """More dense cells than the wavefront-per-cell kernel takes (65,536):
    700k tight clumps of 6 points, some spread over cells that must merge."""
    import paper_2103_05162_amd as fdb
    pts, eps, mp, ref = _many_cells_case()
    _say(f"[gpu] many dense cells: n={len(pts)} K={ref[2]} ({border})")
    if border == "canonical":
        assert_exact(dev, pts, eps, mp, "densebox", ref=ref)
        assert fdb.default_handle(0).last_counts()["dense_cells"] > 65536
        assert_exact(dev, pts, eps, mp, "fdbscan", ref=ref)
    else:
        lab, core, kk = run_gpu(dev, pts, eps, mp, "densebox", border="first")
        assert kk == ref[2]
        assert_tolerance_mode(pts, eps, lab, core, ref[0], ref[1], oracle.check_border)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("d,mp", [(2, 5), (3, 10), (3, 2), (2, 1)])
def test_dbscan_star(dev, algo, d, mp):
    """DBSCAN* (border="none"): canonical clusters, every non-core point noise."""
    pts = _mixture(60 + d + mp, 30011, d, 10, 0.02)
    eps = 0.01 if d == 2 else 0.02
    rl, rc, rk = oracle.dbscan_star(pts, eps, mp)
    lab, core, k = run_gpu(dev, pts, eps, mp, algo, border="none")
    assert k == rk and np.array_equal(core, rc) and np.array_equal(lab, rl)


@pytest.mark.parametrize("algo", ALGOS)
def test_c1_dbscan_star(dev, algo):
    w = workload("c1_blobs2d_16k")
    rl, rc, rk = oracle.dbscan_star(w.points, w.eps, w.min_pts)
    lab, core, k = run_gpu(dev, w.points, w.eps, w.min_pts, algo, border="none")
    assert k == rk and np.array_equal(core, rc) and np.array_equal(lab, rl)


def test_automatic_choice(dev):
    """FDB_ALGO_AUTO runs DenseBox; when the eps grid is too wide for 64-bit keys
    its cells are widened (FDB_INFO_DENSEBOX_FALLBACK); labels exact either way."""
    import paper_2103_05162_amd as fdb
    h = fdb.default_handle(0)
    w = workload("c3_dense3d_8m", 1 / 64)
    assert_exact(dev, w.points, w.eps, w.min_pts, "auto")
    assert not h.last_info() & (fdb.FDB_INFO_AUTO_FDBSCAN | fdb.FDB_INFO_DENSEBOX_FALLBACK)
    assert h.last_counts()["dense_cells"] > 0
    rng = np.random.default_rng(5)
    sparse = rng.uniform(0, 1, size=(60000, 3)).astype(np.float32)
    assert_exact(dev, sparse, 0.02, 5, "auto")
    assert not h.last_info() & fdb.FDB_INFO_DENSEBOX_FALLBACK
    # eps tiny against the extent: the grid cannot be keyed at eps/sqrt(3)
    wide = sparse.copy()
    wide[0] = (1e7, 1e7, 1e7)
    assert_exact(dev, wide, 1e-3, 3, "auto")
    assert h.last_info() & fdb.FDB_INFO_DENSEBOX_FALLBACK
    assert not h.last_info() & fdb.FDB_INFO_AUTO_FDBSCAN


@pytest.mark.parametrize("d", [2, 3])
def test_grid_keyed_in_64_bits(dev, d):
    """A DenseBox grid needing more than 32 key bits (3D: > 1024 cells per axis,
    2D: > 65536) but fitting 64: the device-sized plan picks 64-bit keys and the
    64-bit sort passes; dense clumps and sparse points alike match the oracle."""
    import paper_2103_05162_amd as fdb
    rng = np.random.default_rng(120 + d)
    eps = 4e-4 if d == 3 else 8e-6
    cen = rng.uniform(0, 1, size=(300, d))
    clumps = np.repeat(cen, 40, axis=0) + 0.3 * eps * rng.standard_normal((12000, d))
    pts = np.concatenate([clumps, rng.uniform(0, 1, size=(20000, d))]).astype(np.float32)
    pts = pts[rng.permutation(len(pts))]
    for mp in (2, 5, 30):
        ref = assert_exact(dev, pts, eps, mp, "densebox")
        assert not fdb.default_handle(0).last_info() & fdb.FDB_INFO_DENSEBOX_FALLBACK
        if mp == 5:
            assert fdb.default_handle(0).last_counts()["dense_cells"] > 100
            assert_exact(dev, pts, eps, mp, "fdbscan", ref=ref)


def _boundary_pairs(rng, d, eps, word, mp, count):
    """Pairs (a, b) at distance just inside eps that straddle occupancy-word
    boundaries: "axis" pairs cross one axis's boundary at a random place on the
    other axes, "corner" pairs cross every axis's boundary at once (one pair per
    word corner). Behind each b, away from a, mp - 1 points are packed within
    0.35 eps of b and more than 1.05 eps from a, so b is core and a (2 neighbours)
    is a border point of b's cluster: an a wrongly taken as isolated turns into
    noise and fails the comparison."""
    nw = int(0.9 / word)
    corners = np.stack(np.meshgrid(*[np.arange(1, nw)] * d, indexing="ij"), -1).reshape(-1, d) * word
    ud = np.ones(d) / np.sqrt(d)
    cand = [(c - 0.3 * eps * ud + rng.uniform(-1e-3, 1e-3, size=d) * eps, ud)
            for c in corners[rng.permutation(len(corners))[:count]]]
    for _ in range(20 * count):
        ax = int(rng.integers(0, d))
        u = np.zeros(d)
        u[ax] = 1.0
        a = rng.uniform(0.05, 0.95, size=d)
        a[ax] = rng.integers(1, nw) * word - 0.3 * eps
        cand.append((a, u))
    pairs = []  # pairs kept 3.5 eps apart, so no pair reaches another
    for a, u in cand:
        if len(pairs) < 2 * count and all(np.linalg.norm(a - p[0]) > 3.5 * eps for p in pairs):
            pairs.append((a, u))
    out = []
    for a, u in pairs:
        b = a + eps * (1 - 1e-6) * u
        jit = rng.uniform(-0.05, 0.05, size=(mp - 1, d)) * eps
        pack = b + (0.15 + 0.1 * rng.random((mp - 1, 1))) * eps * u + jit
        out += [a[None], b[None], pack]
    return np.concatenate(out), len(pairs)


@pytest.mark.parametrize("d", [2, 3])
def test_isolated_point_test_edges(dev, d):
    """The DenseBox isolated-point test on its edges: a blob of thousands of
    point primitives (no dense cell at minPts 40) whose runs within one occupancy
    word span many wavefronts; pairs just inside eps straddling word boundaries
    (on one axis, and on every axis at once) whose far partner is core, so their
    near point must come out as a border point; scattered points that are mostly
    alone; and clouds spanning a few grid cells (a one-word map) with core,
    border and noise points in them."""
    rng = np.random.default_rng(70 + d)
    eps = 0.03 if d == 3 else 0.02
    h = eps / np.sqrt(d)              # grid cell side (the bounds below start at 0)
    word = (4 if d == 3 else 8) * h    # side of the cells one occupancy word covers
    blob = 0.5 + rng.uniform(0, 4 * eps, size=(5000 if d == 3 else 3000, d))
    scattered = rng.uniform(0, 1, size=(2000 if d == 3 else 400, d))
    corners = np.array([np.zeros(d), np.ones(d)])
    pts = np.concatenate([blob, scattered, corners]).astype(np.float32)
    rng.shuffle(pts)
    ref = assert_exact(dev, pts, eps, 40, "densebox")
    assert (ref[0] == -1).sum() > 100 and ref[1].sum() > 1000
    for mp in (3, 5):
        pairs, npairs = _boundary_pairs(rng, d, eps, word, mp, 150)
        # scattered points kept 3 eps away from the pairs, so none adds a neighbour
        # to a near point (which would make it core instead of border)
        gap = np.min(np.linalg.norm(scattered[:, None, :] - pairs[None, :, :], axis=2), axis=1)
        pts = np.concatenate([pairs, scattered[gap > 3 * eps], corners]).astype(np.float32)
        # a points sit at rows 0, mp + 1, 2 (mp + 1), ... of `pairs`
        a_rows = np.arange(npairs) * (mp + 1)
        ref = assert_exact(dev, pts, eps, mp, "densebox")
        border = (~ref[1]) & (ref[0] >= 0)
        assert border[a_rows].sum() > 0.7 * npairs, "most near points must be border points"
        assert ref[1][a_rows + 1].all(), "every far partner must be core"
        assert_exact(dev, pts, eps, mp, "fdbscan", ref=ref)
    # one-word maps: a tight core group, a bridge point, a border point 1.2 eps
    # from the group, a noise pair and an isolated point, within 7 cells per axis
    for mp in (2, 3):
        e = np.zeros(d); e[0] = 1.0
        grp = 0.5 * h + rng.uniform(0, 0.02 * eps, size=(5, d))
        bridge = grp[0] + 0.6 * eps * e
        bpt = bridge + 0.6 * eps * e
        far = np.full(d, 6.5 * h)
        pair = np.stack([far - 0.2 * eps * e, far - 0.2 * eps * e - 0.5 * eps * np.roll(e, 1)])
        lone = np.zeros(d); lone[-1] = 6.5 * h
        tiny = np.concatenate([grp, bridge[None], bpt[None], pair, lone[None]]).astype(np.float32)
        ref = assert_exact(dev, tiny, eps, mp, "densebox")
        if mp == 3:
            assert ref[1][:6].all() and not ref[1][6] and ref[0][6] == ref[0][0]
            assert (ref[0][7:] == -1).all()
    dense_tiny = rng.uniform(0, 1.5 * h, size=(40, d)).astype(np.float32)
    ref = assert_exact(dev, dense_tiny, eps, 2, "densebox")
    assert ref[1].all() and ref[2] == 1


@pytest.mark.parametrize("d", [2, 3])
def test_isolated_points_and_pairs_at_eps(dev, d):
    """Isolated points, and pairs at distances a hair inside or outside eps in
    random directions: core, noise and border decisions must be the oracle's bit
    for bit (DenseBox: lone points, records and walks; with minPts 2 a pair is
    core, so a point wrongly taken as isolated by the lone-cell test fails)."""
    rng = np.random.default_rng(40 + d)
    eps, n_single, n_pair = (0.03, 3000, 1500) if d == 3 else (0.02, 150, 100)
    singles = rng.uniform(0, 1, size=(n_single, d))
    a = rng.uniform(0.05, 0.95, size=(n_pair, d))
    u = rng.standard_normal((n_pair, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    scale = eps * rng.choice([1 - 1e-6, 1 - 1e-7, 1.0, 1 + 1e-7, 1 + 1e-6, 0.5, 1.5], size=n_pair)
    pts = np.concatenate([singles, a, a + u * scale[:, None]]).astype(np.float32)
    rng.shuffle(pts)
    for mp in (2, 3, 4):
        ref = assert_exact(dev, pts, eps, mp, "densebox")
        assert (ref[0] == -1).sum() > len(pts) // 10  # plenty of noise
        assert_exact(dev, pts, eps, mp, "fdbscan", ref=ref)
