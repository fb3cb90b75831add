"""GPU kd-tree build vs the oracle build: the permutation, node ranges,
boxes and split dimensions are bit-identical; lambda is an upper bound
(exact to rounding at leaves)."""
import numpy as np
import pytest

from oracle import kdtree as okd
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _gpu_tree(pts, leaf):
    import torch
    from paper_1304_4327_amd import knn
    t = knn.knn_build_tree(torch.from_numpy(pts).cuda(), leaf)
    arr = knn.tree_arrays(t)
    t.close()
    return arr


def _compare(pts, leaf, exact_internal_lambda=False):
    g = _gpu_tree(pts, leaf)
    o = okd.build(pts, leaf)
    assert g["info"]["depth"] == o["depth"]
    assert np.array_equal(g["perm"], o["perm"])
    assert np.array_equal(g["start"], o["start"]) and np.array_equal(g["count"], o["count"])
    live = o["count"] > 0
    assert np.array_equal(g["lo"][live], o["lo"][live])
    assert np.array_equal(g["hi"][live], o["hi"][live])
    assert np.all(g["box_pad"] == 0)
    fl = o["first_leaf"]
    assert np.array_equal(g["split_dim"][:fl], o["split_dim"][:fl])
    assert np.all(g["split_dim"][fl:] == -1)
    # lambda: never below the exact value; leaves within FP32 rounding
    lam_g = g["lam"].astype(np.float64)
    assert np.all(lam_g[live] >= o["lam"][live])
    leaf_live = live.copy()
    leaf_live[:fl] = False
    assert np.all(lam_g[leaf_live] <= o["lam"][leaf_live] * (1 + 2.5e-7) + 1e-30)
    # tree-ordered points are the permuted input, zero padded
    d = pts.shape[1]
    assert np.array_equal(g["points"][:len(pts), :d], pts[g["perm"]])
    assert np.all(g["points"][len(pts):] == 0) and np.all(g["points"][:, d:] == 0)


@pytest.mark.parametrize("n,d,leaf", [(1, 3, 8), (2, 1, 1), (5, 2, 1), (37, 3, 4),
                                      (1000, 3, 20), (4097, 8, 32), (3000, 16, 7),
                                      (2500, 64, 32), (777, 5, 64)])
def test_tree_small(n, d, leaf):
    rng = np.random.default_rng(n + d + leaf)
    pts = rng.standard_normal((n, d)).astype(np.float32)
    _compare(pts, leaf)


@pytest.mark.parametrize("leaf", [1, 3, 32])
def test_tree_with_ties_and_duplicates(leaf):
    rng = np.random.default_rng(leaf)
    pts = rng.integers(0, 4, (3000, 3)).astype(np.float32)
    pts[100:400] = pts[0]
    pts[500:520, 1] = -0.0
    _compare(pts, leaf)


@pytest.mark.parametrize("name,scale", [("gmm1m_d3_k10", 0.12), ("manifold4m_d16_k10", 0.02),
                                        ("manifold1m_d64_k50", 0.03)])
def test_tree_multilevel(name, scale):
    """Sizes that run several grid-wide levels before the per-wave finish."""
    ref, _, _, leaf = datagen.make(name, scale=scale)
    _compare(ref, leaf)


def test_tree_nonfinite_rejected():
    import torch
    from paper_1304_4327_amd import knn
    pts = np.zeros((100, 3), np.float32)
    pts[17, 2] = np.nan
    with pytest.raises(knn.KnnError) as e:
        knn.knn_build_tree(torch.from_numpy(pts).cuda(), 8)
    assert e.value.status == knn.KNN_E_NONFINITE


def test_cached_blocks_reused_across_streams():
    """Trees released on one stream and rebuilt on another (the caching
    allocator hands the same blocks to the new stream after its release
    event) still match the oracle; releasing the cache leaves live trees
    intact."""
    import torch
    from paper_1304_4327_amd import knn
    pts = datagen.uniform(20000, 3, seed=7)
    o = okd.build(pts, 8)
    P = torch.from_numpy(pts).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(3):
        s = s1 if it % 2 == 0 else s2
        with torch.cuda.stream(s):
            t = knn.knn_build_tree(P, 8, stream=s)
            arr = knn.tree_arrays(t)
            t.close()
        assert np.array_equal(arr["perm"], o["perm"])
    assert knn.knn_cached_bytes() > 0
    keep = knn.knn_build_tree(P, 8)
    knn.knn_release_cached_memory()
    assert knn.knn_cached_bytes() == 0
    assert np.array_equal(knn.tree_arrays(keep)["perm"], o["perm"])
    keep.close()


def test_tree_pair_equals_separate_builds():
    """The overlapping pair build gives the same two trees as two calls."""
    import torch
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(30000, 3, seed=11)
    qry = datagen.uniform(17000, 3, seed=12)
    R, Q = torch.from_numpy(ref).cuda(), torch.from_numpy(qry).cuda()
    ta, tb = knn.knn_build_tree_pair(R, Q, 16)
    a, b = knn.tree_arrays(ta), knn.tree_arrays(tb)
    ta.close()
    tb.close()
    for pts, arr in ((ref, a), (qry, b)):
        o = okd.build(pts, 16)
        assert np.array_equal(arr["perm"], o["perm"])
        live = o["count"] > 0
        assert np.array_equal(arr["lo"][live], o["lo"][live])
        assert np.array_equal(arr["hi"][live], o["hi"][live])


@pytest.mark.parametrize("n,d,leaf", [(30000, 3, 16), (2000, 8, 8), (70000, 16, 32), (600, 3, 4)])
def test_tree_pair_equal_sizes(n, d, leaf):
    """Equal sizes, the two builds overlapped: every array equals a separate
    build, bit for bit, and the oracle tree."""
    import torch
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(n, d, seed=31)
    qry = datagen.gmm_pair(n, n, d, 8, seed=32)[1]
    R, Q = torch.from_numpy(ref).cuda(), torch.from_numpy(qry).cuda()
    ta, tb = knn.knn_build_tree_pair(R, Q, leaf)
    pair = (knn.tree_arrays(ta), knn.tree_arrays(tb))
    ta.close()
    tb.close()
    for pts, P in zip((ref, qry), pair):
        t = knn.knn_build_tree(torch.from_numpy(pts).cuda(), leaf)
        S = knn.tree_arrays(t)
        t.close()
        for key in ("points", "perm", "start", "count", "lo", "hi", "lam", "split_dim"):
            live = S["count"] > 0 if key in ("lo", "hi", "lam") else slice(None)
            np.testing.assert_array_equal(P[key][live], S[key][live], err_msg=key)
        o = okd.build(pts, leaf)
        assert np.array_equal(P["perm"], o["perm"])


def test_tree_pair_nonfinite_rejected():
    import torch
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(5000, 3, seed=13)
    qry = datagen.uniform(4000, 3, seed=14)
    qry[123, 1] = np.inf
    with pytest.raises(knn.KnnError) as e:
        knn.knn_build_tree_pair(torch.from_numpy(ref).cuda(), torch.from_numpy(qry).cuda(), 8)
    assert e.value.status == knn.KNN_E_NONFINITE
    # equal sizes, the bad value in either set
    for which in (0, 1):
        a = datagen.uniform(5000, 3, seed=15)
        b = datagen.uniform(5000, 3, seed=16)
        (a, b)[which][77, 2] = np.nan
        with pytest.raises(knn.KnnError) as e:
            knn.knn_build_tree_pair(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), 8)
        assert e.value.status == knn.KNN_E_NONFINITE
