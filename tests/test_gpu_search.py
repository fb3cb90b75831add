"""GPU search vs the FP64 brute-force oracle, element by element, on seeded
inputs shaped like the five workloads (shrunk so the oracle finishes in
seconds, still many tiles and ragged leaves), plus edge cases."""
import numpy as np
import pytest

from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _search(ref, q, k, leaf, bound="B", precision="fp32", leafq=None, stats=False, seed=None):
    torch = _torch()
    from paper_1304_4327_amd import knn
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), leaf)
    if q is None:
        idx, dist, st = knn.knn_search(rt, None, k, bound=bound, precision=precision,
                                       exclude_self=True, stats=stats, seed_radius=seed)
    else:
        qt = knn.knn_build_tree(torch.from_numpy(q).cuda(), leafq or leaf)
        idx, dist, st = knn.knn_search(rt, qt, k, bound=bound, precision=precision, stats=stats,
                                       seed_radius=seed)
        qt.close()
    rt.close()
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), st


def _check(ref, q, k, gi, gd, rows=None):
    self_mode = q is None
    qq = ref if self_mode else q
    if rows is None:
        oi, od = ok.knn(qq, ref, k, exclude_self=self_mode)
    else:
        oi, od = ok.knn_rows(qq, rows, ref, k, exclude_self=self_mode)
    return parity.assert_ok(qq, ref, k, gi, gd, oi, od, rows=rows, exclude_self=self_mode)


def test_figure1_points():
    P = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)
    for k in (1, 2, 3, 4):
        for leaf in (1, 2, 5):
            gi, gd, _ = _search(P, None, k, leaf)
            _check(P, None, k, gi, gd)
    gi, gd, _ = _search(P, None, 4, 2)
    assert gi[0].tolist() == [4, 1, 3, 2]
    np.testing.assert_array_equal(gd[2], np.sqrt(np.float64([4.25, 4.5, 5.0, 6.5])).astype(np.float32))


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
@pytest.mark.parametrize("leaf", [1, 2, 5, 20, 32, 64])
def test_uniform10k_all_knn(bound, leaf):
    ref, _, k, _ = datagen.make("uniform10k_d3_k5")
    gi, gd, st = _search(ref, None, k, leaf, bound=bound, stats=True)
    _check(ref, None, k, gi, gd)
    if bound == "none":
        # no pruning: every pair of the brute force (minus self pairs) is evaluated
        assert st["pairs"] == len(ref) * len(ref)


def test_bound_B_prunes_no_less_than_B1():
    ref, _, k, leaf = datagen.make("uniform10k_d3_k5")
    _, _, sb = _search(ref, None, k, leaf, bound="B", stats=True)
    _, _, s1 = _search(ref, None, k, leaf, bound="B1", stats=True)
    _, _, sn = _search(ref, None, k, leaf, bound="none", stats=True)
    # B is a minimum that includes B1 (allow 1% for the different list
    # evolution a tighter prune causes)
    assert sb["pairs"] <= 1.01 * s1["pairs"]
    assert s1["pairs"] < 0.2 * sn["pairs"]


@pytest.mark.parametrize("name,scale", [("gmm1m_d3_k10", 0.02), ("zipfgmm2m_d8_k10", 0.005),
                                        ("manifold4m_d16_k10", 0.005),
                                        ("manifold1m_d64_k50", 0.01)])
def test_workload_shapes(name, scale):
    ref, q, k, leaf = datagen.make(name, scale=scale)
    gi, gd, _ = _search(ref, q, k, leaf)
    _check(ref, q, k, gi, gd)


@pytest.mark.parametrize("k", [6, 18, 26])
def test_lattice_ties(k):
    g = datagen.lattice(12, 3)
    gi, gd, _ = _search(g, None, k, 8)
    _check(g, None, k, gi, gd)
    inner = np.all((g >= 1) & (g <= 10), axis=1)
    shell = {6: 1.0, 18: 2.0, 26: 3.0}[k]
    np.testing.assert_array_equal(gd[inner, -1], np.float32(np.sqrt(shell)))


def test_duplicates_reported_at_zero():
    rng = np.random.default_rng(3)
    ref = rng.random((2000, 3)).astype(np.float32)
    ref[1000:1100] = ref[5]
    gi, gd, _ = _search(ref, None, 4, 16)
    _check(ref, None, 4, gi, gd)
    assert np.all(gd[1000:1100, 0] == 0)


@pytest.mark.parametrize("m,k", [(2, 1), (9, 8), (70, 64), (300, 1), (300, 64)])
def test_k_edges(m, k):
    rng = np.random.default_rng(m + k)
    ref = rng.random((m, 4)).astype(np.float32)
    q = rng.random((37, 4)).astype(np.float32)
    gi, gd, _ = _search(ref, q, k, 4)
    _check(ref, q, k, gi, gd)


def test_single_query_and_separate_leaf_sizes():
    rng = np.random.default_rng(9)
    ref = rng.random((5000, 3)).astype(np.float32)
    q = rng.random((1, 3)).astype(np.float32)
    gi, gd, _ = _search(ref, q, 7, 32)
    _check(ref, q, 7, gi, gd)
    q = rng.random((999, 3)).astype(np.float32)
    gi, gd, _ = _search(ref, q, 7, 32, leafq=5)
    _check(ref, q, 7, gi, gd)


def test_deterministic():
    ref, q, k, leaf = datagen.make("gmm1m_d3_k10", scale=0.01)
    a = _search(ref, q, k, leaf)
    b = _search(ref, q, k, leaf)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_k_too_large_rejected():
    torch = _torch()
    from paper_1304_4327_amd import knn
    ref = np.random.default_rng(0).random((10, 3)).astype(np.float32)
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), 4)
    with pytest.raises(knn.KnnError) as e:
        knn.knn_search(rt, None, 10, exclude_self=True)
    assert e.value.status == knn.KNN_E_INVALID_ARG


@pytest.mark.parametrize("name,scale", [("manifold4m_d16_k10", 0.005), ("manifold1m_d64_k50", 0.01)])
@pytest.mark.parametrize("bound", ["B", "B1"])
def test_bf16_tiles_match_oracle(name, scale, bound):
    """BF16 MFMA tiles with the proven margin and FP64 re-score: the same
    exact answer as the oracle."""
    ref, q, k, leaf = datagen.make(name, scale=scale)
    gi, gd, st = _search(ref, q, k, leaf, bound=bound, precision="bf16", stats=True)
    _check(ref, q, k, gi, gd)


@pytest.mark.parametrize("d,k", [(9, 1), (16, 7), (24, 10), (32, 15), (20, 32), (33, 20), (64, 64)])
def test_bf16_dims_and_self(d, k):
    rng = np.random.default_rng(d * 100 + k)
    ref = (rng.standard_normal((3000, d)) * rng.uniform(0.1, 3.0, d)).astype(np.float32)
    ref[100:140] = ref[7]          # duplicates: zero distances, ties
    kk = min(k, 63)
    gi, gd, _ = _search(ref, None, kk, 16, precision="bf16")
    _check(ref, None, kk, gi, gd)
    q = rng.standard_normal((500, d)).astype(np.float32)
    gi, gd, _ = _search(ref, q, k, 32, precision="bf16")
    _check(ref, q, k, gi, gd)


@pytest.mark.parametrize("d,k,leaf", [(12, 5, 20), (30, 4, 24), (17, 11, 9), (32, 16, 32)])
def test_bf16_matrix_core_traversal_shapes(d, k, leaf):
    """The traversal kernel with matrix-core tiles (stride 16 or 32, lists of
    <= 16) at leaf sizes below 32 (rows past the leaf, idle lanes of a half)
    and every list length it instantiates, in query and self mode."""
    rng = np.random.default_rng(d * 1000 + k * 10 + leaf)
    basis = rng.standard_normal((5, d))
    ref = (rng.random((6000, 5)) @ basis + 0.03 * rng.standard_normal((6000, d))).astype(np.float32)
    q = (rng.random((900, 5)) @ basis + 0.03 * rng.standard_normal((900, d))).astype(np.float32)
    gi, gd, _ = _search(ref, q, k, leaf, precision="bf16")
    _check(ref, q, k, gi, gd)
    gi, gd, _ = _search(ref, None, k, leaf, precision="bf16")
    _check(ref, None, k, gi, gd)


@pytest.mark.parametrize("n_ref,n_q,k,leaf", [(20, 5, 7, 32), (700, 5, 7, 32), (700, 70, 3, 16),
                                             (3000, 200, 50, 32)])
def test_bf16_sweep_small_and_idle_waves(n_ref, n_q, k, leaf):
    """d = 64 leaf sweep at shapes that reach its edges: one reference leaf
    (only the flush after the sweep multiplies a tile), workgroups whose
    four query leaves are not all present (idle waves still stage and meet
    at every barrier), and lists of 50 with many kept leaves."""
    rng = np.random.default_rng(n_ref + 7 * n_q + k)
    basis = rng.standard_normal((6, 64))
    ref = (rng.random((n_ref, 6)) @ basis + 0.05 * rng.standard_normal((n_ref, 64))).astype(np.float32)
    q = (rng.random((n_q, 6)) @ basis + 0.05 * rng.standard_normal((n_q, 64))).astype(np.float32)
    kk = min(k, n_ref - 1)
    gi, gd, _ = _search(ref, q, kk, leaf, precision="bf16")
    _check(ref, q, kk, gi, gd)
    for bound in ("B1", "none"):
        gi2, gd2, _ = _search(ref, q, kk, leaf, bound=bound, precision="bf16")
        assert np.array_equal(gi, gi2) and np.array_equal(gd, gd2)


@pytest.mark.parametrize("d", [16, 32])
def test_bf16_same_answer_as_fp32(d):
    """Stride 16 and 32 with lists of <= 16 run the traversal kernel with
    matrix-core tiles: every list equals the FP32 kernel's bit for bit and
    passes the oracle check."""
    if d == 16:
        ref, q, k, leaf = datagen.make("manifold4m_d16_k10", scale=0.004)
    else:
        rng = np.random.default_rng(32)
        basis = rng.standard_normal((8, 32))
        ref = (rng.random((20000, 8)) @ basis + 0.02 * rng.standard_normal((20000, 32))).astype(np.float32)
        q = (rng.random((3000, 8)) @ basis + 0.02 * rng.standard_normal((3000, 32))).astype(np.float32)
        k, leaf = 10, 32
    a = _search(ref, q, k, leaf, precision="fp32")
    b = _search(ref, q, k, leaf, precision="bf16")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    _check(ref, q, k, b[0], b[1])


def test_bf16_low_dim_unsupported():
    torch = _torch()
    from paper_1304_4327_amd import knn
    ref = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), 8)
    with pytest.raises(knn.KnnError) as e:
        knn.knn_search(rt, None, 3, exclude_self=True, precision="bf16")
    assert e.value.status == knn.KNN_E_UNSUPPORTED


# ---- the whole path in one call (knn_all_knn) --------------------------------
def _all_knn(ref, q, k, leaf, precision="fp32", stats=False):
    torch = _torch()
    from paper_1304_4327_amd import knn
    R = torch.from_numpy(ref).cuda()
    Q = None if q is None else torch.from_numpy(q).cuda()
    idx, dist, st = knn.knn_all_knn(R, Q, k, leaf, precision=precision, exclude_self=q is None,
                                    stats=stats)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), st


@pytest.mark.parametrize("name,scale", [("gmm1m_d3_k10", 0.03), ("manifold4m_d16_k10", 0.0075)])
def test_all_knn_matches_oracle_and_separate_calls(name, scale):
    """One call (both builds, search) equals the separate calls bit for bit
    and passes the oracle check."""
    ref, q, k, leaf = datagen.make(name, scale=scale)
    gi, gd, st = _all_knn(ref, q, k, leaf, stats=True)
    si, sd, _ = _search(ref, q, k, leaf)
    np.testing.assert_array_equal(gi, si)
    np.testing.assert_array_equal(gd, sd)
    _check(ref, q, k, gi, gd)
    assert st["ms_ref_build"] > 0 and st["ms_query_build"] > 0 and st["pairs"] > 0


def test_all_knn_self_mode():
    ref, _, k, leaf = datagen.make("uniform10k_d3_k5")
    gi, gd, st = _all_knn(ref, None, k, leaf, stats=True)
    si, sd, _ = _search(ref, None, k, leaf)
    np.testing.assert_array_equal(gi, si)
    np.testing.assert_array_equal(gd, sd)
    _check(ref, None, k, gi, gd)
    assert st["ms_query_build"] == 0


def test_all_knn_bf16():
    ref, q, k, leaf = datagen.make("manifold4m_d16_k10", scale=0.005)
    gi, gd, _ = _all_knn(ref, q, k, leaf, precision="bf16")
    _check(ref, q, k, gi, gd)


@pytest.mark.parametrize("which", ["ref", "query"])
def test_all_knn_nonfinite_rejected(which):
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(6000, 3, seed=21)
    qry = datagen.uniform(3000, 3, seed=22)
    (ref if which == "ref" else qry)[77, 2] = np.nan
    with pytest.raises(knn.KnnError) as e:
        _all_knn(ref, qry, 4, 16)
    assert e.value.status == knn.KNN_E_NONFINITE


def test_all_knn_rejects_k_too_large():
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(50, 3, seed=23)
    qry = datagen.uniform(40, 3, seed=24)
    with pytest.raises(knn.KnnError) as e:
        _all_knn(ref, qry, 50, 8)
    assert e.value.status == knn.KNN_E_INVALID_ARG


def test_binding_rejects_wrong_output_shapes():
    torch = _torch()
    from paper_1304_4327_amd import knn
    ref = datagen.uniform(500, 3, 4)
    rt = knn.knn_build_tree(torch.from_numpy(ref).cuda(), 8)
    nl = rt.info()["n_leaves"]
    good = (torch.empty((500, 4), dtype=torch.int64, device="cuda"),
            torch.empty((500, 4), dtype=torch.float32, device="cuda"))
    for bad in [(good[0][:499], good[1]), (good[0], good[1].double()),
                (good[0].t().contiguous().t(), good[1])]:
        with pytest.raises(ValueError):
            knn.knn_search(rt, None, 4, exclude_self=True, out=bad)
    with pytest.raises(ValueError):
        knn.knn_search(rt, None, 4, exclude_self=True,
                       seed_radius=torch.zeros(nl - 1, device="cuda"))
    with pytest.raises(ValueError):
        knn.knn_search(rt, None, 4, exclude_self=True,
                       leaf_kth_out=torch.zeros(nl, dtype=torch.float64, device="cuda"))
    knn.knn_search(rt, None, 4, exclude_self=True, out=good)
