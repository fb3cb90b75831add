"""k-furthest neighbours on the GPU (knn_search_furthest, the inverted rules
of the closing remark of Section "k-Nearest Neighbor Search") against the
FP64 oracle, element by element: Figure 1, every bound, several leaf sizes,
the workload shapes at reduced size (many tiles, ragged leaves), ties on a
lattice, duplicates, k at its limits, and pruning that actually prunes."""
import numpy as np
import pytest

from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _far(ref, q, k, leaf, bound="B", stats=False):
    import torch
    from paper_1304_4327_amd import knn
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = None if q is None else knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    idx, dist, st = knn.knn_search_furthest(rt, qt, k, bound=bound, exclude_self=q is None,
                                            stats=stats)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), st


def _check(ref, q, k, gi, gd, rows=None):
    self_mode = q is None
    qq = ref if self_mode else q
    rows_ = np.arange(len(qq)) if rows is None else rows
    oi, od = ok.furthest_rows(qq, rows_, ref, k, exclude_self=self_mode)
    return parity.assert_ok_furthest(qq, ref, k, gi, gd, oi, od, rows=rows,
                                     exclude_self=self_mode)


def test_figure1_points():
    P = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)
    for k in (1, 2, 3, 4):
        for leaf in (1, 2, 5):
            gi, gd, _ = _far(P, None, k, leaf)
            _check(P, None, k, gi, gd)
    gi, gd, _ = _far(P, None, 4, 2)
    assert gi[0].tolist() == [2, 3, 1, 4]
    np.testing.assert_array_equal(gd[2], np.sqrt(np.float64([6.5, 5.0, 4.5, 4.25])).astype(np.float32))


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
@pytest.mark.parametrize("leaf", [1, 5, 20, 32, 64])
def test_uniform10k_all_kfn(bound, leaf):
    ref, _, k, _ = datagen.make("uniform10k_d3_k5")
    gi, gd, st = _far(ref, None, k, leaf, bound=bound, stats=True)
    _check(ref, None, k, gi, gd)
    if bound == "none":
        assert st["pairs"] == len(ref) * len(ref)


def test_bound_prunes():
    ref, _, k, leaf = datagen.make("uniform10k_d3_k5")
    sb = _far(ref, None, k, leaf, bound="B", stats=True)[2]
    s1 = _far(ref, None, k, leaf, bound="B1", stats=True)[2]
    sn = _far(ref, None, k, leaf, bound="none", stats=True)[2]
    assert sb["pairs"] <= 1.01 * s1["pairs"] and s1["pairs"] < 0.2 * sn["pairs"]


@pytest.mark.parametrize("name,scale", [("gmm1m_d3_k10", 0.02), ("zipfgmm2m_d8_k10", 0.005),
                                        ("manifold4m_d16_k10", 0.005),
                                        ("manifold1m_d64_k50", 0.01)])
def test_workload_shapes(name, scale):
    ref, q, k, leaf = datagen.make(name, scale=scale)
    gi, gd, _ = _far(ref, q, k, leaf)
    _check(ref, q, k, gi, gd)


@pytest.mark.parametrize("k", [1, 8, 20])
def test_lattice_ties(k):
    g = datagen.lattice(9, 3)
    gi, gd, _ = _far(g, None, k, 8)
    _check(g, None, k, gi, gd)


def test_duplicates_and_full_lists():
    """References at distance 0 still fill a list when fewer than k others
    are farther; k = m - 1 returns every other point."""
    ref = np.zeros((40, 3), np.float32)
    ref[:3] = [[1, 0, 0], [0, 2, 0], [0, 0, 3]]
    gi, gd, _ = _far(ref, None, 5, 4)
    _check(ref, None, 5, gi, gd)
    assert (gd[5:, 3:] == 0).all()
    rng = np.random.default_rng(4)
    small = rng.random((30, 2)).astype(np.float32)
    gi, gd, _ = _far(small, None, 29, 4)
    _check(small, None, 29, gi, gd)


@pytest.mark.parametrize("m,k", [(2, 1), (70, 64), (300, 1), (300, 63)])
def test_k_edges(m, k):
    rng = np.random.default_rng(m + k)
    ref = rng.random((m, 4)).astype(np.float32)
    q = rng.random((37, 4)).astype(np.float32)
    gi, gd, _ = _far(ref, q, k, 4)
    _check(ref, q, k, gi, gd)


def test_full_size_sampled_rows():
    """1M x 1M, d = 3, k = 10 at full size: a seeded sample of 2^12 rows
    against the oracle."""
    ref, q, k, leaf = datagen.make("gmm1m_d3_k10")
    gi, gd, st = _far(ref, q, k, leaf, stats=True)
    print(f"furthest 1M x 1M: {st['pairs'] / len(q):.0f} pairs/query, "
          f"{st['ms_search']:.2f} ms", flush=True)
    rows = np.sort(np.random.default_rng(5).choice(len(q), 4096, replace=False))
    _check(ref, q, k, gi, gd, rows=rows)
    assert (np.diff(gd, axis=1) <= 0).all()
