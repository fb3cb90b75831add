"""The acceptance predicate accepts the oracle's own answer and rejects each
kind of planted mistake (planted in a copy of the oracle's answer, on the
CPU)."""
import numpy as np
import pytest

from oracle import knn as ok
from oracle import parity
from paper_1304_4327_amd import datagen


@pytest.fixture(scope="module")
def case():
    ref, q, k, _ = datagen.make("gmm1m_d3_k10", scale=0.002)
    idx, d2 = ok.knn(q, ref, k)
    return q, ref, k, idx, d2


def _run(case, gi, gd):
    q, ref, k, idx, d2 = case
    return parity.check(q, ref, k, gi, gd, idx, d2)[0]


def test_accepts_oracle_answer(case):
    q, ref, k, idx, d2 = case
    f = _run(case, idx, np.sqrt(d2).astype(np.float32))
    assert not any(f.values())


@pytest.mark.parametrize("mistake", ["swap_far", "duplicate", "bad_distance", "unsorted",
                                     "out_of_range"])
def test_rejects_planted_mistakes(case, mistake):
    q, ref, k, idx, d2 = case
    gi = idx.copy()
    gd = np.sqrt(d2).astype(np.float32)
    if mistake == "swap_far":
        gi[3, 0] = int(ok.knn(q[3:4], ref, 200)[0][0, -1])   # a far reference
        key = "missing_neighbour"
    elif mistake == "duplicate":
        gi[4, 1] = gi[4, 0]
        key = "duplicates"
    elif mistake == "bad_distance":
        gd[5, 2] *= 1.0 + 5e-5
        key = "distance_error"
    elif mistake == "unsorted":
        gd[6, [0, 1]] = gd[6, [1, 0]] + np.array([1e-3, 0], np.float32)
        key = "unsorted"
    else:
        gi[7, 3] = len(ref)
        key = "out_of_range"
    f = _run(case, gi, gd)
    assert f[key] >= 1


def test_excuses_exact_ties():
    """Equal distances at the k-th place: either index is acceptable."""
    x = np.array([[0, 0], [1, 0], [0, 1], [5, 5]], np.float32)
    idx, d2 = ok.knn(x, x, 1, exclude_self=True)
    alt = idx.copy()
    alt[0, 0] = 2 if idx[0, 0] == 1 else 1
    f, _ = parity.check(x, x, 1, alt, np.sqrt(d2), idx, d2, exclude_self=True)
    assert not any(f.values())
    f, _ = parity.check(x, x, 1, np.array([[0], [0], [0], [0]]), np.sqrt(d2), idx, d2,
                        exclude_self=True)
    assert f["self_match"] >= 1


def test_rejects_beyond_kth_inside_a_tie():
    """A tie at the k-th place hides a planted far entry from the
    missing-neighbour test (neither tied point is required), so only the
    upper-bound test can see it: query 0 has neighbours 1 and 2 at distance
    1 (a tie at k = 1) and 3 at distance 2."""
    x = np.array([[0, 0], [1, 0], [0, 1], [2, 0], [5, 5]], np.float32)
    idx, d2 = ok.knn(x, x, 1, exclude_self=True)
    gi = idx.copy()
    gd = np.sqrt(d2).astype(np.float32)
    gi[0, 0] = 3
    gd[0, 0] = 2.0
    f, _ = parity.check(x, x, 1, gi, gd, idx, d2, exclude_self=True)
    assert f["missing_neighbour"] == 0
    assert f["beyond_kth"] == 1
    assert sum(f.values()) == 1
