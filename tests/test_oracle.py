"""Pins for the CPU oracle, against facts fixed by the paper and by mathematics
rather than by the oracle itself:

* hand-built point sets whose clustering follows from the definitions of
  Section 2.1 (core, border, noise; closed eps-ball including the point);
* the bridging hazard of Section 3.2 (a border point between two clusters
  must not join them);
* the minPts = 2 special case of Section 2.1, which is the connected
  components of the eps-graph (scipy's graph routine);
* minPts = 1 (every point is core) and other degenerate cases;
* an independent library DBSCAN (scikit-learn) on inputs where no pair lies
  near the threshold, so fp64 and fp32 distance tests agree;
* the two neighbour-enumeration modes against each other;
* exact invariances of the fp32 test (reflection, axis swap, 2^k scaling).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph
import sklearn.cluster

import oracle
from tests.helpers import partition_map, pick_safe_eps, same_partition

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- the distance test -------------------------------------------------------

def test_pred_closed_ball_exact_values():
    # 3-4-5 triangle scaled by 1/8: 0.375^2 + 0.5^2 = 0.625^2 holds exactly in fp32.
    assert oracle.pred([0.0, 0.0], [0.375, 0.5], 0.625)
    # the next fp32 above 0.5 makes the squared distance exceed eps^2 by 2^-24
    q = [0.375, float(np.nextafter(np.float32(0.5), np.float32(1)))]
    assert not oracle.pred([0.0, 0.0], q, 0.625)
    # 3D: (1,2,2)/4 has length 3/4 exactly.
    assert oracle.pred([0, 0, 0], [0.25, 0.5, 0.5], 0.75)
    assert not oracle.pred([0, 0, 0], [0.25, 0.5, 0.5], float(np.nextafter(np.float32(0.75), np.float32(0))))
    # a point is in its own neighbourhood, even for the smallest positive eps
    assert oracle.pred([1.5, -2.0, 3.0], [1.5, -2.0, 3.0], float(np.float32(1e-30)))


def test_pred_symmetric_and_matches_exact_distance_off_threshold():
    rng = np.random.default_rng(11)
    for d in (2, 3):
        p = rng.uniform(-1, 1, size=(400, d)).astype(np.float32)
        q = rng.uniform(-1, 1, size=(400, d)).astype(np.float32)
        eps = 0.7
        exact = np.sqrt(((p.astype(np.float64) - q.astype(np.float64)) ** 2).sum(1))
        for i in range(len(p)):
            a = oracle.pred(p[i], q[i], eps)
            assert a == oracle.pred(q[i], p[i], eps)
            if abs(exact[i] - eps) > 1e-5:
                assert a == (exact[i] <= eps)


# ---- hand-built sets -----------------------------------------------------------

def test_two_lines_noise_and_border():
    # eps=1, minPts=3. Line A (spacing 0.5) and line B are all core; (3,0) has
    # itself and (2,0) at distance exactly 1 -> count 2, border of A; (5,5) is noise.
    A = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    B = [(10, 0), (10.5, 0), (11, 0)]
    pts = np.array(A + B + [(5, 5), (3, 0)], dtype=np.float32)
    labels, core, k = oracle.dbscan(pts, 1.0, 3, "brute")
    assert k == 2
    assert core.tolist() == [True] * 8 + [False, False]
    assert labels.tolist() == [0] * 5 + [1] * 3 + [-1, 0]
    counts = oracle.neighbor_counts(pts, 1.0, "brute")
    assert counts.tolist() == [3, 4, 5, 4, 4, 3, 3, 3, 1, 2]


def test_dbscan_star_drops_border_points():
    # DBSCAN* (Section 2.1): same sets as test_two_lines_noise_and_border, but the
    # border point (3,0) is noise, like (5,5); clusters and ids are unchanged.
    A = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    B = [(10, 0), (10.5, 0), (11, 0)]
    pts = np.array(A + B + [(5, 5), (3, 0)], dtype=np.float32)
    labels, core, k = oracle.dbscan_star(pts, 1.0, 3, "brute")
    assert k == 2
    assert labels.tolist() == [0] * 5 + [1] * 3 + [-1, -1]
    # the bridging configuration: b, (5.75,0) and (0,0) are border points, all noise
    B2 = [(3.75, 0), (4.25, 0), (4.75, 0), (5.25, 0), (5.75, 0)]
    A2 = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    pts = np.array(B2 + A2 + [(2.875, 0)], dtype=np.float32)
    labels, core, k = oracle.dbscan_star(pts, 1.0, 4, "brute")
    assert k == 2
    assert labels.tolist() == [0, 0, 0, 0, -1, -1, 1, 1, 1, 1, -1]


def test_bridging_border_point_does_not_merge_clusters():
    # eps=1, minPts=4 (Section 3.2's bridging hazard); all coordinates dyadic, so
    # every distance is exact. b=(2.875,0) is within eps of core (2,0) of cluster A
    # and of core (3.75,0) of cluster B but has only 3 neighbours itself, so A and
    # B stay apart; b takes the smaller id.
    B = [(3.75, 0), (4.25, 0), (4.75, 0), (5.25, 0), (5.75, 0)]
    A = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    pts = np.array(B + A + [(2.875, 0)], dtype=np.float32)
    labels, core, k = oracle.dbscan(pts, 1.0, 4, "brute")
    assert k == 2
    # B: 3.75, 4.25, 4.75, 5.25 core; 5.75 border.  A: 0 border; 0.5..2 core.  b border.
    assert core.tolist() == [True, True, True, True, False, False, True, True, True, True, False]
    assert labels.tolist() == [0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0]


def test_lattice_counts_and_core_interior():
    # unit lattice, eps=1: interior points have 5 neighbours (self + 4), edges 4, corners 3
    g = np.stack(np.meshgrid(np.arange(6), np.arange(5), indexing="ij"), -1).reshape(-1, 2).astype(np.float32)
    counts = oracle.neighbor_counts(g, 1.0, "brute")
    x, y = g[:, 0], g[:, 1]
    on_x = (x == 0) | (x == 5)
    on_y = (y == 0) | (y == 4)
    expect = np.where(on_x & on_y, 3, np.where(on_x | on_y, 4, 5))
    assert np.array_equal(counts, expect)
    labels, core, k = oracle.dbscan(g, 1.0, 5, "brute")
    assert np.array_equal(core, expect == 5)
    assert k == 1
    # every edge point touches an interior core point except the 4 corners
    assert np.array_equal(labels == -1, on_x & on_y)


def test_degenerate_inputs():
    empty = np.zeros((0, 3), np.float32)
    labels, core, k = oracle.dbscan(empty, 0.1, 3)
    assert k == 0 and labels.size == 0
    one = np.array([[0.25, 0.5, 0.75]], np.float32)
    assert oracle.dbscan(one, 0.1, 1)[0].tolist() == [0]
    assert oracle.dbscan(one, 0.1, 2)[0].tolist() == [-1]
    dup = np.full((50, 2), 0.3, np.float32)
    labels, core, k = oracle.dbscan(dup, 1e-6, 50)
    assert k == 1 and core.all() and (labels == 0).all()
    labels, core, k = oracle.dbscan(dup, 1e-6, 51)
    assert k == 0 and (labels == -1).all()


def test_min_pts_one_every_point_is_core():
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 1, size=(300, 3)).astype(np.float32)
    eps = pick_safe_eps(pts, 0.08)
    labels, core, k = oracle.dbscan(pts, eps, 1, "brute")
    assert core.all()
    comps = _fp64_components(pts, eps)
    assert same_partition(labels, comps)
    assert k == comps.max() + 1


def test_eps_larger_than_diameter_is_one_cluster_and_tiny_eps_all_noise():
    rng = np.random.default_rng(6)
    pts = rng.uniform(0, 1, size=(500, 2)).astype(np.float32)
    labels, core, k = oracle.dbscan(pts, 2.0, 10)
    assert k == 1 and core.all() and (labels == 0).all()
    labels, core, k = oracle.dbscan(pts, 1e-7, 2)
    assert k == 0 and (labels == -1).all() and not core.any()


# ---- minPts = 2 is connected components of the eps-graph ----------------------

def _fp64_components(pts, eps):
    p = pts.astype(np.float64)
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
    adj = scipy.sparse.csr_matrix(d <= eps)
    return scipy.sparse.csgraph.connected_components(adj, directed=False)[1]


@pytest.mark.parametrize("dim", [2, 3])
def test_min_pts_two_is_connected_components(dim):
    rng = np.random.default_rng(20 + dim)
    pts = rng.uniform(0, 1, size=(700, dim)).astype(np.float32)
    eps = pick_safe_eps(pts, 0.04 if dim == 2 else 0.09)
    labels, core, k = oracle.dbscan(pts, eps, 2, "brute")
    comps = _fp64_components(pts, eps)
    sizes = np.bincount(comps)
    single = sizes[comps] == 1
    assert np.array_equal(core, ~single)
    assert np.array_equal(labels == -1, single)
    assert same_partition(labels, comps, ~single)
    assert k == int((sizes > 1).sum())


# ---- an independent library DBSCAN ---------------------------------------------

def _blobs(rng, n, dim, k, sigma):
    c = rng.uniform(0, 1, size=(k, dim))
    lab = rng.integers(0, k + 1, size=n)
    pts = np.where(lab[:, None] < k, c[np.minimum(lab, k - 1)] + sigma * rng.standard_normal((n, dim)),
                   rng.uniform(0, 1, size=(n, dim)))
    return pts.astype(np.float32)


@pytest.mark.parametrize("dim,min_pts,seed", [(2, 5, 1), (3, 4, 2), (2, 10, 3), (3, 3, 4)])
def test_matches_sklearn_dbscan(dim, min_pts, seed):
    rng = np.random.default_rng(seed)
    pts = _blobs(rng, 1500, dim, 6, 0.03)
    eps = pick_safe_eps(pts, 0.03 if dim == 2 else 0.06)
    labels, core, k = oracle.dbscan(pts, eps, min_pts, "brute")
    sk = sklearn.cluster.DBSCAN(eps=eps, min_samples=min_pts, algorithm="brute").fit(pts.astype(np.float64))
    sk_core = np.zeros(len(pts), bool)
    sk_core[sk.core_sample_indices_] = True
    assert np.array_equal(core, sk_core)
    assert np.array_equal(labels == -1, sk.labels_ == -1)
    m = partition_map(labels, sk.labels_, core)
    assert m is not None and len(m) == k
    # scikit-learn gives a border point to the first cluster that reaches it;
    # both choices must be clusters holding a core point within eps.
    assert oracle.check_border(pts, eps, core, labels) == 0
    assert oracle.check_border(pts, eps, core, sk.labels_) == 0
    # some border points exist, so the border rule was exercised
    assert ((~core) & (labels >= 0)).sum() > 0


# ---- the border checker must catch wrong border labels ---------------------------
#
# check_border is the only judge of first-claim outputs (Section 3.2: a border
# point joins whichever cluster claims it first), so it is pinned here on labels
# known to be wrong: each planted violation must be counted exactly once, and the
# valid alternatives of the bridging case must pass.

def _two_lines():
    # the set of test_two_lines_noise_and_border: eps = 1, minPts = 3; points 0-4
    # line A (core), 5-7 line B (core), 8 = (5,5) noise, 9 = (3,0) border of A only
    A = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    B = [(10, 0), (10.5, 0), (11, 0)]
    return np.array(A + B + [(5, 5), (3, 0)], dtype=np.float32)


@pytest.mark.parametrize("method", ["brute", "grid"])
def test_check_border_counts_planted_violations(method):
    pts = _two_lines()
    labels, core, k = oracle.dbscan(pts, 1.0, 3, "brute")
    assert labels.tolist() == [0] * 5 + [1] * 3 + [-1, 0]
    assert oracle.check_border(pts, 1.0, core, labels, method) == 0
    # a labelled non-core point whose label's cores are all beyond eps
    # (B's nearest core (10,0) is 7 away from (3,0))
    bad = labels.copy(); bad[9] = 1
    assert oracle.check_border(pts, 1.0, core, bad, method) == 1
    # a noise label on a point with a core within eps ((2,0) at distance exactly 1)
    bad = labels.copy(); bad[9] = -1
    assert oracle.check_border(pts, 1.0, core, bad, method) == 1
    # a cluster label on a point with no core neighbour at all
    bad = labels.copy(); bad[8] = 0
    assert oracle.check_border(pts, 1.0, core, bad, method) == 1
    # an id that names no cluster
    bad = labels.copy(); bad[9] = 7
    assert oracle.check_border(pts, 1.0, core, bad, method) == 1
    # the three at once are three violations
    bad = labels.copy(); bad[9] = 1; bad[8] = 0
    assert oracle.check_border(pts, 1.0, core, bad, method) == 2
    bad[9] = -1
    assert oracle.check_border(pts, 1.0, core, bad, method) == 2
    # core points' labels are not the checker's business (the partition test is)
    bad = labels.copy(); bad[0] = 1
    assert oracle.check_border(pts, 1.0, core, bad, method) == 0


@pytest.mark.parametrize("method", ["brute", "grid"])
def test_check_border_accepts_either_cluster_of_a_bridging_point(method):
    # the bridging set of test_bridging_border_point_does_not_merge_clusters:
    # b = (2.875, 0) is within eps of a core of each cluster, so both ids are valid
    # and noise is not; (5.75, 0) reaches only B and (0, 0) only A.
    B = [(3.75, 0), (4.25, 0), (4.75, 0), (5.25, 0), (5.75, 0)]
    A = [(0, 0), (0.5, 0), (1, 0), (1.5, 0), (2, 0)]
    pts = np.array(B + A + [(2.875, 0)], dtype=np.float32)
    labels, core, k = oracle.dbscan(pts, 1.0, 4, "brute")
    for b_label, expect in ((0, 0), (1, 0), (-1, 1), (2, 1)):
        lab = labels.copy(); lab[10] = b_label
        assert oracle.check_border(pts, 1.0, core, lab, method) == expect, b_label
    lab = labels.copy(); lab[4] = 1   # (5.75, 0) moved to A: A's nearest core (2,0) is 3.75 away
    assert oracle.check_border(pts, 1.0, core, lab, method) == 1
    lab = labels.copy(); lab[5] = 0   # (0, 0) moved to B
    assert oracle.check_border(pts, 1.0, core, lab, method) == 1


@pytest.mark.parametrize("dim,min_pts,seed", [(2, 5, 1), (3, 4, 2)])
def test_check_border_catches_one_moved_sklearn_border_point(dim, min_pts, seed):
    """scikit-learn's own labels (an independent implementation) pass; moving one
    border point into a cluster none of whose cores is within eps (decided in fp64
    on an eps with no pair near the threshold) gives exactly one violation, and
    turning one border point into noise gives exactly one."""
    rng = np.random.default_rng(seed)
    pts = _blobs(rng, 1500, dim, 6, 0.03)
    eps = pick_safe_eps(pts, 0.03 if dim == 2 else 0.06)
    sk = sklearn.cluster.DBSCAN(eps=eps, min_samples=min_pts, algorithm="brute").fit(pts.astype(np.float64))
    core = np.zeros(len(pts), bool)
    core[sk.core_sample_indices_] = True
    lab = sk.labels_.astype(np.int32)
    assert oracle.check_border(pts, eps, core, lab) == 0
    p = pts.astype(np.float64)
    border = np.flatnonzero(~core & (lab >= 0))
    assert border.size > 0
    i = int(border[0])
    near = np.sqrt(((p - p[i]) ** 2).sum(1)) <= eps
    reachable = set(lab[near & core].tolist())
    far = [c for c in range(lab.max() + 1) if c not in reachable]
    assert far
    moved = lab.copy(); moved[i] = far[0]
    assert oracle.check_border(pts, eps, core, moved) == 1
    assert oracle.check_border(pts, eps, core, moved, "brute") == 1
    dropped = lab.copy(); dropped[i] = -1
    assert oracle.check_border(pts, eps, core, dropped) == 1
    # a noise point given a cluster: noise has no core within eps, so any id is wrong
    noise = np.flatnonzero(lab < 0)
    assert noise.size > 0
    given = lab.copy(); given[int(noise[0])] = 0
    assert oracle.check_border(pts, eps, core, given) == 1


# ---- brute vs grid enumeration ------------------------------------------------

@pytest.mark.parametrize("dim,n,eps,min_pts,seed", [
    (2, 3000, 0.02, 5, 7), (3, 3000, 0.05, 4, 8), (3, 2500, 0.04, 2, 9), (2, 2000, 0.03, 1, 10),
])
def test_grid_mode_equals_brute_mode(dim, n, eps, min_pts, seed):
    rng = np.random.default_rng(seed)
    pts = _blobs(rng, n, dim, 5, 0.02)
    a = oracle.dbscan(pts, eps, min_pts, "brute")
    b = oracle.dbscan(pts, eps, min_pts, "grid")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    assert np.array_equal(oracle.neighbor_counts(pts, eps, "brute"), oracle.neighbor_counts(pts, eps, "grid"))


def test_grid_mode_keeps_pairs_at_cell_boundaries():
    # pairs at distance exactly eps along each axis, straddling the cells
    eps = 0.25
    base = np.array([[0.0, 0.0, 0.0]], np.float32)
    pts = np.concatenate([base, base + [eps, 0, 0], base + [0, eps, 0], base + [0, 0, eps],
                          base + [2 * eps, 0, 0], base + [3 * eps, 0, 0]]).astype(np.float32)
    a = oracle.neighbor_counts(pts, eps, "brute")
    b = oracle.neighbor_counts(pts, eps, "grid")
    assert a.tolist() == [4, 3, 2, 2, 3, 2]
    assert np.array_equal(a, b)


# ---- exact invariances ------------------------------------------------------------

def test_reflection_axis_swap_and_power_of_two_scaling_are_exact():
    rng = np.random.default_rng(31)
    pts = _blobs(rng, 2000, 3, 6, 0.02)
    eps, mp = 0.03, 5
    ref = oracle.dbscan(pts, eps, mp, "grid")
    cases = [(lambda p: -p, 1.0), (lambda p: p[:, [1, 0, 2]], 1.0),
             (lambda p: p * np.float32(2.0 ** 7), 2.0 ** 7), (lambda p: p * np.float32(2.0 ** -9), 2.0 ** -9)]
    for t, f in cases:
        q = np.ascontiguousarray(t(pts)).astype(np.float32)
        got = oracle.dbscan(q, float(np.float32(eps)) * f, mp, "grid")
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_permutation_changes_only_names():
    rng = np.random.default_rng(32)
    pts = _blobs(rng, 2500, 2, 6, 0.02)
    eps, mp = 0.02, 6
    labels, core, k = oracle.dbscan(pts, eps, mp)
    perm = rng.permutation(len(pts))
    l2, c2, k2 = oracle.dbscan(pts[perm], eps, mp)
    assert k2 == k
    assert np.array_equal(c2, core[perm])
    assert np.array_equal(l2 == -1, labels[perm] == -1)
    assert same_partition(l2, labels[perm], c2)
    assert oracle.check_border(pts[perm], eps, c2, l2) == 0


# ---- stored values from the oracle's own committed script ------------------------

def test_golden_summaries_match():
    """Summaries of the full-size workloads written by tests/golden/make_golden.py
    (which calls only the oracle); recomputed here on the reduced C1 case."""
    path = os.path.join(GOLDEN, "c1_blobs2d_16k.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    g = json.load(open(path))
    from workloads.gen import workload
    w = workload("c1_blobs2d_16k")
    labels, core, k = oracle.dbscan(w.points, w.eps, w.min_pts)
    assert k == g["num_clusters"]
    assert int(core.sum()) == g["num_core"]
    assert int((labels == -1).sum()) == g["num_noise"]


def test_neighbors_of_matches_counts():
    rng = np.random.default_rng(41)
    pts = rng.uniform(0, 1, size=(3000, 3)).astype(np.float32)
    counts = oracle.neighbor_counts(pts, 0.08, "brute")
    for i in (0, 17, 2999):
        nb = oracle.neighbors_of(pts, 0.08, i)
        assert len(nb) == counts[i] and i in nb
        assert all(oracle.pred(pts[i], pts[j], 0.08) for j in nb)
