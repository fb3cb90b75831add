"""Pins for the reading of the k-NN bound B(N_q) (Section "k-Nearest
Neighbor Search"): the literal dual-tree traversal with the safe reading and
a strict prune reaches the brute-force answer; the printed recursion and the
printed non-strict comparison do not always."""
import numpy as np
import pytest

from oracle import dualtree as dt
from oracle import knn as ok
from oracle import kdtree as kd


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 30))
    d = int(rng.integers(1, 4))
    k = int(rng.integers(1, 4))
    ls = int(rng.integers(1, 5))
    x = rng.random((n, d)).astype(np.float32)
    return x, k, ls


def _exact(x, k, ls, bound, strict=True):
    oi, od = ok.knn_numpy(x, x, k, exclude_self=True)
    t = dt.DualTreeKNN(x, x, k, leaf_size=ls, bound=bound, exclude_self=True, strict=strict)
    N, D = t.run()
    return np.allclose(D ** 2, od, rtol=1e-12, atol=1e-14), t


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
def test_safe_bounds_are_exact(bound):
    """Correctness argument (after Algorithm 3): a valid bound never prunes
    a needed subtree, so the result equals brute force."""
    for seed in range(120):
        x, k, ls = _case(seed)
        ok_, _ = _exact(x, k, ls, bound)
        assert ok_, seed


def test_pruning_actually_prunes():
    rng = np.random.default_rng(5)
    x = rng.random((300, 2)).astype(np.float32)
    ok_b, tb = _exact(x, 3, 4, "B")
    ok_n, tn = _exact(x, 3, 4, "none")
    assert ok_b and ok_n
    assert tb.base_cases < 0.5 * tn.base_cases


def test_B_never_looser_than_B1_visits():
    """B is a minimum that includes B1, so it never visits more pairs."""
    for seed in range(40):
        x, k, ls = _case(seed)
        _, tb = _exact(x, k, ls, "B")
        _, t1 = _exact(x, k, ls, "B1")
        assert tb.base_cases <= t1.base_cases


def test_nonstrict_prune_loses_a_neighbour():
    """Seed 25: a point at exactly the bound min D[k] + 2 lambda (inherited
    from the parent) is the true k-th neighbour; pruning at d_min >= B drops
    it, pruning at d_min > B keeps it."""
    x, k, ls = _case(25)
    assert not _exact(x, k, ls, "B", strict=False)[0]
    assert _exact(x, k, ls, "B", strict=True)[0]


def test_printed_recursion_is_not_a_bound():
    """With the exact final k-th distances, the printed recursion (child
    term B(N_c) + 2(lambda_q - lambda_c)) falls below the largest true k-th
    distance of some node's descendants on these seeded inputs; the safe
    reading never does (it is an upper bound by the triangle inequality)."""
    found = 0
    for seed in range(200):
        rng = np.random.default_rng(1000 + seed)
        n = int(rng.integers(6, 40))
        d = int(rng.integers(1, 4))
        k = int(rng.integers(1, 4))
        ls = int(rng.integers(1, 5))
        x = rng.random((n, d)).astype(np.float32)
        if seed % 2:
            x[: n // 2] = (0.5 + 0.01 * rng.random((n // 2, d))).astype(np.float32)
        _, od = ok.knn_numpy(x, x, k, exclude_self=True)
        kth = np.sqrt(od[:, k - 1])
        t = kd.build(x, ls)
        printed, safe, need = dt.printed_bound_bottom_up(t, kth)
        live = t["count"] > 0
        assert np.all(safe[live] >= need[live] * (1 - 1e-12))
        if np.any(printed[live] < need[live] * (1 - 1e-9)):
            found += 1
    assert found > 0


def test_printed_recursion_loses_neighbours_in_traversal():
    bad = 0
    for seed in range(300):
        x, k, ls = _case(seed)
        bad += not _exact(x, k, ls, "printed")[0]
    assert bad > 0
