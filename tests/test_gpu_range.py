"""Range search on the GPU (knn_range_count / knn_range_fill, Section "Range
Search", Algorithms 5 and 6) against the FP64 oracle.  The in-range decision
is taken the same way on both sides (FP64 squared distance, products
rounded, against the FP64 squares of the ends), so the neighbour sets must
be identical, query by query; distances are FP32 of the FP64 value."""
import numpy as np
import pytest

from oracle import knn as ok
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu

FIG1 = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)


def _range(ref, q, lo, hi, leaf, bound="B", stats=False):
    import torch
    from paper_1304_4327_amd import knn
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    qt = None if q is None else knn.knn_build_tree(torch.from_numpy(q).cuda(), leaf)
    off, idx, dist, st = knn.knn_range_search(rt, qt, lo, hi, bound=bound,
                                              exclude_self=q is None, stats=stats)
    torch.cuda.synchronize()
    return off.cpu().numpy(), idx.cpu().numpy(), dist.cpu().numpy(), st


def _check(ref, q, lo, hi, got, rows=None):
    """Per query: the same index set as the oracle; each distance equal to
    FP32 of the FP64 distance."""
    off, idx, dist = got[:3]
    qq = ref if q is None else q
    rows = np.arange(len(qq)) if rows is None else rows
    oo, oi, od2 = ok.range_rows(qq, rows, ref, lo, hi, exclude_self=q is None)
    for t, row in enumerate(rows):
        gi = idx[off[row]:off[row + 1]]
        gd = dist[off[row]:off[row + 1]]
        order = np.argsort(gi)
        want = oi[oo[t]:oo[t + 1]]
        assert np.array_equal(gi[order], want), f"row {row}"
        np.testing.assert_array_equal(gd[order], np.sqrt(od2[oo[t]:oo[t + 1]]).astype(np.float32))
    return int(oo[-1])


@pytest.mark.parametrize("lo,hi", [(0.6, 1.5), (0.5, 1.5), (0.0, 0.0), (0.0, 10.0), (5.0, 6.0)])
@pytest.mark.parametrize("leaf", [1, 2, 5])
def test_figure1(lo, hi, leaf):
    got = _range(FIG1, None, lo, hi, leaf)
    _check(FIG1, None, lo, hi, got)


@pytest.mark.parametrize("bound", ["B", "none"])
@pytest.mark.parametrize("leaf", [1, 7, 20, 64])
def test_uniform10k(bound, leaf):
    ref, _, _, _ = datagen.make("uniform10k_d3_k5")
    got = _range(ref, None, 0.01, 0.05, leaf, bound=bound, stats=True)
    total = _check(ref, None, 0.01, 0.05, got)
    assert total > 0
    cnt_st = got[3][0]
    assert cnt_st["inserts"] == total
    if bound == "none":
        assert cnt_st["pairs"] == len(ref) * len(ref)
    else:
        assert cnt_st["pairs"] < 0.1 * len(ref) * len(ref)


def _typical(ref, q, k=10):
    """A range around the workload's typical 10-th neighbour distance."""
    rows = np.arange(0, len(q), max(1, len(q) // 64))
    _, d2 = ok.knn_rows(q, rows, ref, k)
    m = float(np.median(np.sqrt(d2[:, -1])))
    return 0.5 * m, 1.2 * m


@pytest.mark.parametrize("name,scale", [("gmm1m_d3_k10", 0.02), ("zipfgmm2m_d8_k10", 0.005),
                                        ("manifold4m_d16_k10", 0.005),
                                        ("manifold1m_d64_k50", 0.01)])
def test_workload_shapes(name, scale):
    ref, q, _, leaf = datagen.make(name, scale=scale)
    lo, hi = _typical(ref, q)
    got = _range(ref, q, lo, hi, leaf)
    assert _check(ref, q, lo, hi, got) > len(q)


@pytest.mark.parametrize("lo,hi,count", [(1.0, 1.0, 6), (1.0, np.sqrt(2.0) + 1e-12, 18),
                                         (np.sqrt(2.0) - 1e-12, np.sqrt(3.0) + 1e-12, 20),
                                         (0.0, np.sqrt(3.0) + 1e-12, 26)])
def test_lattice_shells(lo, hi, count):
    g = datagen.lattice(10, 3)
    off, idx, dist, _ = _range(g, None, lo, hi, 8)
    inner = np.all((g >= 1) & (g <= 8), axis=1)
    assert np.all(np.diff(off)[inner] == count)
    _check(g, None, lo, hi, (off, idx, dist))


def test_duplicates_empty_and_everything():
    rng = np.random.default_rng(3)
    ref = rng.random((3000, 3)).astype(np.float32)
    ref[1000:1100] = ref[5]
    got = _range(ref, None, 0.0, 0.0, 16)          # exact duplicates only
    _check(ref, None, 0.0, 0.0, got)
    assert got[0][-1] == 101 * 100                 # each of the 101 copies sees 100 others
    got = _range(ref, None, 5.0, 6.0, 16)          # nothing that far
    assert got[0][-1] == 0
    q = rng.random((50, 3)).astype(np.float32)
    got = _range(ref, q, 0.0, 2.0, 16)             # every pair
    assert got[0][-1] == 50 * 3000
    _check(ref, q, 0.0, 2.0, got)


def test_full_size_sampled_rows():
    """1M x 1M, d = 3, radius 0.2 at full size: 2^12 seeded rows against the
    oracle, the offsets checked whole."""
    ref, q, _, leaf = datagen.make("gmm1m_d3_k10")
    lo, hi = 0.0, 0.2
    got = _range(ref, q, lo, hi, leaf, stats=True)
    off = got[0]
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(got[1])
    st = got[3]
    print(f"range 1M x 1M: {off[-1] / len(q):.1f} neighbours/query, count "
          f"{st[0]['ms_search']:.2f} ms + fill {st[1]['ms_search']:.2f} ms, "
          f"{st[0]['pairs'] / len(q):.0f} pairs/query", flush=True)
    rows = np.sort(np.random.default_rng(6).choice(len(q), 4096, replace=False))
    _check(ref, q, lo, hi, got, rows=rows)
