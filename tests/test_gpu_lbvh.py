"""The LBVH build and the masked walk of the main phase, pinned to the paper's
Figure 1 (Section 4.1): eight leaves with 4-bit codes 0000, 0001, 0100, 0101,
1000, 1100, 1101, 1110 give the tree drawn there (root 0 -> 3, 4; 3 -> 1, 2;
4 -> leaf 4, 5; 5 -> 6, leaf 7; 6 -> leaf 5, leaf 6), and the walk of thread 4
reaches exactly leaves 5, 6, 7."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    import paper_2103_05162_amd as fdb
    return fdb.default_handle(0)


def test_figure1_tree_and_mask(h):
    codes = [0b0000, 0b0001, 0b0100, 0b0101, 0b1000, 0b1100, 0b1101, 0b1110]
    gamma, other, leaves = h.debug_lbvh(codes, mask=4)
    # internal node k covers [min(k, other), max(k, other)] split after gamma:
    # children are node gamma (or leaf gamma) and node gamma+1 (or leaf gamma+1)
    ranges = {k: (min(k, o), max(k, o), g) for k, (o, g) in enumerate(zip(other, gamma))}
    assert ranges[0] == (0, 7, 3)      # root: internal 3 = [0,3], internal 4 = [4,7]
    assert ranges[3] == (0, 3, 1)      # internal 1 = [0,1], internal 2 = [2,3]
    assert ranges[4] == (4, 7, 4)      # leaf 4, internal 5 = [5,7]
    assert ranges[5] == (5, 7, 6)      # internal 6 = [5,6], leaf 7
    assert ranges[6] == (5, 6, 5)      # leaves 5 and 6
    assert ranges[1] == (0, 1, 0) and ranges[2] == (2, 3, 2)
    assert leaves.tolist() == [5, 6, 7]
    _, _, all_leaves = h.debug_lbvh(codes, mask=-1)
    assert all_leaves.tolist() == list(range(8))


@pytest.mark.parametrize("seed", range(6))
def test_masked_walk_reaches_exactly_the_leaves_above_the_mask(h, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 3000))
    bits = int(rng.integers(1, 40))
    keys = np.sort(rng.integers(0, 2 ** bits, size=m, dtype=np.uint64))
    for leaf in (1, 4, 32):
        for mask in sorted({-1, 0, m // 3, m - 2, m - 1, int(rng.integers(0, m))}):
            _, _, leaves = h.debug_lbvh(keys, mask=mask, leaf_size=leaf)
            assert leaves.tolist() == list(range(mask + 1, m)), (m, bits, leaf, mask)


def _prefix(keys, m, i, j):
    # common-prefix length of sorted keys i and j (64-bit), equal keys told apart by index
    if j < 0 or j >= m:
        return -1
    a, b = int(keys[i]), int(keys[j])
    if a == b:
        return 64 + 32 - (i ^ j).bit_length()
    return 64 - (a ^ b).bit_length()


def _karras_top_down(keys):
    """Karras' rule for internal node i (range direction, extent by doubling and
    binary search, split by binary search), written out from the definition."""
    m = len(keys)
    other, gamma = [], []
    for i in range(m - 1):
        dl, dr = _prefix(keys, m, i, i - 1), _prefix(keys, m, i, i + 1)
        d = 1 if dr > dl else -1
        dmin = min(dl, dr)
        lmax = 2
        while _prefix(keys, m, i, i + lmax * d) > dmin:
            lmax *= 2
        l, t = 0, lmax // 2
        while t >= 1:
            if _prefix(keys, m, i, i + (l + t) * d) > dmin:
                l += t
            t //= 2
        j = i + l * d
        dnode = _prefix(keys, m, i, j)
        s, t = 0, l
        while True:
            t = (t + 1) // 2
            if _prefix(keys, m, i, i + (s + t) * d) > dnode:
                s += t
            if t <= 1:
                break
        other.append(j)
        gamma.append(i + s * d + (-1 if d < 0 else 0))
    return other, gamma


@pytest.mark.parametrize("seed", range(8))
def test_hierarchy_equals_karras_top_down(h, seed):
    """The bottom-up build gives Karras' tree and numbering exactly, across many
    256-leaf workgroups, with duplicate keys and with few distinct keys."""
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(2, 6000)) if seed < 6 else (257 if seed == 6 else 4096)
    bits = int(rng.integers(1, 48))
    keys = np.sort(rng.integers(0, 2 ** bits, size=m, dtype=np.uint64))
    gamma, other, _ = h.debug_lbvh(keys, mask=-1)
    o_ref, g_ref = _karras_top_down(keys.tolist())
    assert np.asarray(other).tolist() == o_ref
    assert np.asarray(gamma).tolist() == g_ref
