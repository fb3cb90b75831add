"""Pins of the k-furthest-neighbour oracle (closing remark of Section
"k-Nearest Neighbor Search"): Figure 1's points with hand-computed lists,
the defining k-subset property on tiny inputs, closed forms on a lattice,
the numpy form, the literal inverted dual-tree search, and the acceptance
predicate on planted mistakes."""
import itertools
import os

import numpy as np
import pytest

from oracle import dualtree as dt
from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen

FIG1 = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)


def _golden(golden_dir):
    idx, d2 = [], []
    for line in open(os.path.join(golden_dir, "fig1_allkfn.txt")):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        pairs = [p.split() for p in line.split(":", 1)[1].split(",")]
        idx.append([int(a) for a, _ in pairs])
        d2.append([float(b) for _, b in pairs])
    return np.array(idx), np.array(d2)


def test_figure1_furthest_lists(golden_dir):
    gi, gd2 = _golden(golden_dir)
    oi, od2 = ok.furthest(FIG1, FIG1, 4, exclude_self=True)
    np.testing.assert_array_equal(oi, gi)
    np.testing.assert_array_equal(od2, gd2)


def test_numpy_form_agrees():
    rng = np.random.default_rng(3)
    for n, m, d, k in [(30, 40, 3, 5), (17, 17, 2, 16), (50, 60, 8, 1)]:
        q = rng.random((n, d)).astype(np.float32)
        r = rng.random((m, d)).astype(np.float32)
        a = ok.furthest(q, r, k)
        b = ok.furthest_numpy(q, r, k)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_allclose(a[1], b[1], rtol=1e-15)   # summation order


def test_k_subset_property_exhaustive():
    """For n <= 9 every k-subset is enumerated: the oracle's set is one
    whose smallest distance is at least every excluded distance, and no
    subset has a larger sum of squared distances."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        n = int(rng.integers(3, 10))
        x = rng.integers(0, 4, (n, 2)).astype(np.float32)   # many ties
        k = int(rng.integers(1, n - 1))
        oi, od2 = ok.furthest(x, x, k, exclude_self=True)
        for i in range(n):
            d2 = ((x.astype(np.float64) - x[i]) ** 2).sum(1)
            others = [j for j in range(n) if j != i]
            chosen = set(oi[i].tolist())
            assert len(chosen) == k and i not in chosen
            excl = [d2[j] for j in others if j not in chosen]
            if excl:
                assert d2[list(chosen)].min() >= max(excl)
            best = max(sum(d2[list(s)]) for s in itertools.combinations(others, k))
            assert d2[list(chosen)].sum() == best


def test_lattice_closed_form():
    g = datagen.lattice(3, 3) - 1.0          # {-1, 0, 1}^3
    centre = int(np.nonzero((g == 0).all(1))[0][0])
    corner = int(np.nonzero((g == 1).all(1))[0][0])
    oi, od2 = ok.furthest(g, g, 8, exclude_self=True)
    assert set(oi[centre].tolist()) == {i for i in range(27) if (np.abs(g[i]) == 1).all()}
    np.testing.assert_array_equal(od2[centre], np.full(8, 3.0))
    # from (1,1,1) a coordinate -1, 0 or 1 adds 4, 1 or 0: the opposite
    # corner (12), then two -1 and a 0 (9, three points), then two -1 and a
    # 1 (8, three points)
    assert (g[oi[corner, 0]] == -1).all() and od2[corner, 0] == 12.0
    np.testing.assert_array_equal(od2[corner, 1:7], [9.0] * 3 + [8.0] * 3)


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 30))
    d = int(rng.integers(1, 4))
    k = int(rng.integers(1, 4))
    ls = int(rng.integers(1, 5))
    return rng.random((n, d)).astype(np.float32), k, ls


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
def test_literal_dual_tree_furthest_is_exact(bound):
    """The inverted rules reach the brute-force answer under every bound."""
    for seed in range(120):
        x, k, ls = _case(seed)
        t = dt.DualTreeKFN(x, x, k, leaf_size=ls, bound=bound, exclude_self=True)
        _, D = t.run()
        _, od2 = ok.furthest_numpy(x, x, k, exclude_self=True)
        assert np.allclose(D ** 2, od2, rtol=1e-12, atol=1e-14), seed


def test_literal_dual_tree_furthest_prunes():
    rng = np.random.default_rng(5)
    x = rng.random((300, 2)).astype(np.float32)
    tb = dt.DualTreeKFN(x, x, 3, leaf_size=4, bound="B", exclude_self=True)
    tb.run()
    tn = dt.DualTreeKFN(x, x, 3, leaf_size=4, bound="none", exclude_self=True)
    tn.run()
    assert tb.base_cases < 0.5 * tn.base_cases


@pytest.mark.parametrize("mistake", ["swap_near", "tie_beyond", "duplicate", "bad_distance",
                                     "unsorted"])
def test_furthest_predicate(mistake):
    ref, q, k, _ = datagen.make("gmm1m_d3_k10", scale=0.002)
    oi, od2 = ok.furthest(q, ref, k)
    gi, gd = oi.copy(), np.sqrt(od2).astype(np.float32)
    f, _ = parity.check_furthest(q, ref, k, gi, gd, oi, od2)
    assert not any(f.values())
    if mistake == "swap_near":
        gi[3, 0] = int(ok.knn(q[3:4], ref, 1)[0][0, 0])     # the nearest reference
        key = "missing_neighbour"
    elif mistake == "duplicate":
        gi[4, 1] = gi[4, 0]
        key = "duplicates"
    elif mistake == "bad_distance":
        gd[5, 2] *= 1.0 + 5e-5
        key = "distance_error"
    elif mistake == "unsorted":
        gd[6, [0, 1]] = gd[6, [1, 0]] - np.array([1e-3, 0], np.float32)
        key = "unsorted"
    else:
        # a tie at the k-th place hides a planted near entry from the
        # missing-neighbour test: only the lower-bound test sees it
        x = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [-5, -5]], np.float32)
        xi, xd2 = ok.furthest(x, x, 2, exclude_self=True)     # query 0: 4 (50), then 1 / 2 tie
        bi, bd = xi.copy(), np.sqrt(xd2).astype(np.float32)
        bi[0, 1], bd[0, 1] = 3, 0.5
        f, _ = parity.check_furthest(x, x, 2, bi, bd, xi, xd2, exclude_self=True)
        assert f["missing_neighbour"] == 0 and f["beyond_kth"] == 1
        return
    f, _ = parity.check_furthest(q, ref, k, gi, gd, oi, od2)
    assert f[key] >= 1
