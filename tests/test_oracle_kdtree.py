"""Pins for the oracle kd-tree: every property of the split rule is checked
directly on the output, without re-running the build's own logic."""
import numpy as np
import pytest

from oracle import kdtree as kd


def _check(pts, t):
    n, d = pts.shape
    L, ls = t["depth"], t["leaf_size"]
    # depth: smallest L with ceil(n / 2^L) <= leaf size
    assert -(-n // (1 << L)) <= ls
    assert L == 0 or -(-n // (1 << (L - 1))) > ls
    perm = t["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    fl = t["first_leaf"]
    for node in range(t["n_nodes"]):
        s, c = int(t["start"][node]), int(t["count"][node])
        idx = perm[s:s + c]
        # a leaf lists its points in ascending original index
        if node >= fl:
            assert np.all(np.diff(idx) > 0)
        if c:
            # tight box containing the points (Definition 1: convex set
            # containing the node's points)
            assert np.array_equal(t["lo"][node], pts[idx].min(0))
            assert np.array_equal(t["hi"][node], pts[idx].max(0))
            # lambda: max distance from the centre to a descendant point
            dist = np.sqrt(((pts[idx].astype(np.float64) - t["centre"][node]) ** 2).sum(1))
            assert t["lam"][node] == dist.max()
        if node >= fl:
            assert c <= ls
            continue
        a, b = 2 * node + 1, 2 * node + 2
        # children partition the parent's range, left gets floor(c/2)
        assert t["count"][a] == c // 2 and t["count"][b] == c - c // 2
        assert t["start"][a] == s and t["start"][b] == s + c // 2
        if c == 0:
            continue
        j = t["split_dim"][node]
        ext = (t["hi"][node] - t["lo"][node]).astype(np.float32)
        assert ext[j] == ext.max() and np.all(ext[:j] < ext[j])
        # left keys (coordinate, index) all precede right keys
        la, lb = perm[s:s + c // 2], perm[s + c // 2:s + c]
        if la.size and lb.size:
            kl = max(zip(pts[la, j].tolist(), la.tolist()))
            kr = min(zip(pts[lb, j].tolist(), lb.tolist()))
            assert kl < kr
        # children's boxes lie inside the parent's
        for ch in (a, b):
            if t["count"][ch]:
                assert np.all(t["lo"][ch] >= t["lo"][node])
                assert np.all(t["hi"][ch] <= t["hi"][node])


@pytest.mark.parametrize("n,d,ls", [(1, 3, 4), (5, 2, 1), (37, 3, 4), (200, 3, 20),
                                    (1000, 8, 32), (333, 16, 7), (64, 1, 2)])
def test_tree_properties_random(n, d, ls):
    rng = np.random.default_rng(n * 31 + d)
    pts = rng.standard_normal((n, d)).astype(np.float32)
    _check(pts, kd.build(pts, ls))


@pytest.mark.parametrize("ls", [1, 2, 3, 5])
def test_tree_properties_with_ties(ls):
    """Integer coordinates and duplicate points: ties on the split
    coordinate are broken by original index."""
    rng = np.random.default_rng(11)
    pts = rng.integers(0, 3, (90, 3)).astype(np.float32)
    pts[10:20] = pts[0]
    _check(pts, kd.build(pts, ls))


def test_widest_dimension_tie_goes_to_lowest():
    pts = np.array([[0, 0], [1, 1], [2, 2], [3, 3]], np.float32)
    t = kd.build(pts, 2)
    assert t["split_dim"][0] == 0
    assert t["perm"].tolist() == [0, 1, 2, 3]


def test_leaf_of_rows_inverts_perm():
    rng = np.random.default_rng(3)
    pts = rng.random((100, 3)).astype(np.float32)
    t = kd.build(pts, 8)
    lr = kd.leaf_of_rows(t)
    fl = t["first_leaf"]
    for i in range(100):
        node = fl + lr[i]
        s, c = t["start"][node], t["count"][node]
        assert i in t["perm"][s:s + c]
