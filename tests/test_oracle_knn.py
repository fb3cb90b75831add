"""Pins for the FP64 brute-force oracle against facts the paper and the
mathematics fix, independent of the oracle's own code."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import knn as ok
from paper_1304_4327_amd import datagen


def _read_fig1(golden_dir):
    pts, rows = {}, {}
    with open(os.path.join(golden_dir, "fig1_allknn.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("P "):
                _, i, x, y = line.split()
                pts[int(i)] = (float(x), float(y))
            elif line.startswith("N "):
                head, tail = line[2:].split(":", 1)
                q = int(head)
                rows[q] = [(int(a), float(b)) for a, b in (t.split(":") for t in tail.split())]
    P = np.array([pts[i] for i in range(len(pts))], np.float32)
    return P, rows


def test_figure1_all_knn(golden_dir):
    """Figure 1 (Section "Space Trees") points: the hand-computed lists,
    including the exact ties (x4, x5 for x2; x1, x4 for x5) ordered by
    index."""
    P, rows = _read_fig1(golden_dir)
    idx, d2 = ok.knn(P, P, 4, exclude_self=True)
    for q, lst in rows.items():
        assert idx[q].tolist() == [a for a, _ in lst]
        assert d2[q].tolist() == [b for _, b in lst]


def test_figure1_numpy_form_agrees(golden_dir):
    P, rows = _read_fig1(golden_dir)
    idx, d2 = ok.knn_numpy(P, P, 4, exclude_self=True)
    for q, lst in rows.items():
        assert idx[q].tolist() == [a for a, _ in lst]


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_subset_property(seed):
    """For tiny sets enumerate every k-subset S and check the defining
    property of the k nearest neighbours: the returned set is one whose
    largest distance does not exceed the smallest distance outside it, and
    no other subset has a smaller sorted distance vector."""
    rng = np.random.default_rng(seed)
    n, m, d = 4, 9, int(rng.integers(1, 4))
    q = rng.integers(0, 4, (n, d)).astype(np.float32)     # integer grid: many ties
    r = rng.integers(0, 4, (m, d)).astype(np.float32)
    for k in (1, 3, 5):
        idx, d2 = ok.knn(q, r, k)
        for i in range(n):
            dist = ((q[i].astype(np.float64) - r.astype(np.float64)) ** 2).sum(1)
            best = None
            for S in itertools.combinations(range(m), k):
                key = (sorted(dist[list(S)]), sorted(S))
                if best is None or key < best:
                    best = key
            got = sorted(idx[i].tolist())
            assert sorted(dist[got]) == best[0]
            # lexicographic tie-break by index selects the smallest index set
            assert got == best[1]
            assert d2[i].tolist() == sorted(dist[got])


def test_self_exclusion_by_index_only():
    """The footnote to the k-NN BaseCase: a point does not return itself;
    an exact duplicate under another index is still a neighbour (at 0)."""
    x = np.array([[0, 0], [0, 0], [3, 0], [0, 4]], np.float32)
    idx, d2 = ok.knn(x, x, 2, exclude_self=True)
    assert idx[0].tolist() == [1, 2] and d2[0].tolist() == [0.0, 9.0]
    assert idx[1].tolist() == [0, 2]
    assert idx[3].tolist() == [0, 1] and d2[3].tolist() == [16.0, 16.0]


@pytest.mark.parametrize("d", [2, 3])
def test_lattice_closed_form(d):
    """Interior points of an integer grid: the 2d face neighbours at 1, then
    the edge neighbours at sqrt(2), then (d = 3) the corners at sqrt(3)."""
    side = 6
    g = datagen.lattice(side, d)
    inner = np.all((g >= 1) & (g <= side - 2), axis=1)
    qrows = np.where(inner)[0]
    shells = {2: [(4, 1.0), (4, 2.0)], 3: [(6, 1.0), (12, 2.0), (8, 3.0)]}[d]
    k_total = 0
    for count, dist2 in shells:
        k_total += count
        idx, d2 = ok.knn_rows(g, qrows, g, k_total, exclude_self=True)
        assert np.all(d2[:, k_total - count:] == dist2)
        assert np.all(d2[:, :k_total - count] < dist2)
        off = g[idx] - g[qrows][:, None, :]
        assert np.all(np.abs(off) <= 1)


def test_against_scipy_kdtree():
    """Cross-check with an independent library routine (scipy cKDTree,
    FP64, exact search) on continuous data, where ties have probability 0."""
    scipy_spatial = pytest.importorskip("scipy.spatial")
    ref, q, k, _ = datagen.make("gmm1m_d3_k10", scale=0.004)
    idx, d2 = ok.knn(q, ref, k)
    tree = scipy_spatial.cKDTree(ref.astype(np.float64))
    dd, ii = tree.query(q.astype(np.float64), k=k)
    assert np.array_equal(ii, idx)
    np.testing.assert_allclose(np.sqrt(d2), dd, rtol=1e-12)


def test_rows_variant_matches_full():
    ref, q, k, _ = datagen.make("manifold1m_d64_k50", scale=0.002)
    idx, d2 = ok.knn(q, ref, k)
    rows = np.array([0, 5, len(q) - 1])
    idx2, d22 = ok.knn_rows(q, rows, ref, k)
    assert np.array_equal(idx[rows], idx2) and np.array_equal(d2[rows], d22)


def test_numpy_and_c_agree_on_random():
    rng = np.random.default_rng(7)
    q = rng.random((40, 5)).astype(np.float32)
    r = rng.random((70, 5)).astype(np.float32)
    a = ok.knn(q, r, 7)
    b = ok.knn_numpy(q, r, 7)
    assert np.array_equal(a[0], b[0]) and np.allclose(a[1], b[1], rtol=0, atol=1e-15)


def test_invalid_k_rejected():
    x = np.zeros((3, 2), np.float32)
    with pytest.raises(ValueError):
        ok.knn(x, x, 3)          # needs k < m
    with pytest.raises(ValueError):
        ok.knn(x, x, 0)


def test_uniform_mean_knn_distance_sanity():
    """Statistical sanity only (not parity): for N uniform points in the unit
    cube the mean k-th neighbour distance of interior points is close to
    Gamma(k + 1/3) / Gamma(k) * (N * 4 pi / 3)^(-1/3)."""
    ref, _, k, _ = datagen.make("uniform10k_d3_k5")
    idx, d2 = ok.knn(ref, ref, k, exclude_self=True)
    inner = np.all((ref > 0.1) & (ref < 0.9), axis=1)
    got = np.sqrt(d2[inner, k - 1]).mean()
    want = math.gamma(k + 1 / 3) / math.gamma(k) * (len(ref) * 4 * math.pi / 3) ** (-1 / 3)
    assert abs(got / want - 1) < 0.03
