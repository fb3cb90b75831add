"""Acceptance predicate: does a GPU k-NN answer match the FP64 oracle?

Per query, with delta_k the oracle's k-th distance and delta_r the FP64
distance of any reference r:

* the returned index set G has k distinct in-range entries and, with the self
  match excluded, does not contain the query's own index;
* {r : delta_r < delta_k (1 - tol_set)}  is a subset of  G, and
  G is a subset of {r : delta_r <= delta_k (1 + tol_set)}  -- the sets are
  identical unless the oracle has distances within tol_set of delta_k
  (equal distances have no defined order in the paper's BaseCase, which
  inserts only on a strict improvement);
* each returned distance is within tol_dist relative of delta_r, and exactly
  0 when delta_r is 0;
* returned distances are non-decreasing (the lists are ordered by distance).

tol_set = 1e-6 and tol_dist = 1e-5 are the acceptance tolerances of the
search, fixed up front for every precision mode.
"""
from __future__ import annotations

import numpy as np

from . import knn as _knn

TOL_SET = 1e-6
TOL_DIST = 1e-5


def check(q, r, k, gpu_idx, gpu_dist, ora_idx, ora_d2, rows=None,
          exclude_self=False, tol_set=TOL_SET, tol_dist=TOL_DIST):
    """Return a dict of failure counts (all zero on success) and details.

    ``rows`` are the query rows the oracle arrays describe (default: all);
    ``gpu_idx``/``gpu_dist`` are full-size GPU outputs, indexed by row.
    """
    q = np.asarray(q, np.float32)
    r = np.asarray(r, np.float32)
    m = r.shape[0]
    n = q.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, np.int64)
    gi = np.asarray(gpu_idx)[rows].astype(np.int64)
    gd = np.asarray(gpu_dist)[rows].astype(np.float64)
    oi = np.asarray(ora_idx, np.int64)
    od2 = np.asarray(ora_d2, np.float64)
    assert gi.shape == (len(rows), k) and oi.shape == gi.shape

    fails = {}
    in_range = (gi >= 0) & (gi < m)
    fails["out_of_range"] = int((~in_range).sum())
    gi_safe = np.where(in_range, gi, 0)
    srt = np.sort(gi_safe, axis=1)
    fails["duplicates"] = int((srt[:, 1:] == srt[:, :-1]).any(axis=1).sum()) if k > 1 else 0
    if exclude_self:
        fails["self_match"] = int((gi == rows[:, None]).any(axis=1).sum())
    else:
        fails["self_match"] = 0

    # FP64 distance of every returned reference
    qi = np.repeat(rows, k)
    d2_g = _knn.pair_d2(q, r, qi, gi_safe.ravel()).reshape(len(rows), k)
    delta_g = np.sqrt(d2_g)
    delta_o = np.sqrt(od2)
    dk = delta_o[:, k - 1:k]

    upper = delta_g <= dk * (1.0 + tol_set)
    fails["beyond_kth"] = int((~upper & in_range).any(axis=1).sum())

    must = delta_o < dk * (1.0 - tol_set)
    missing = np.zeros(len(rows), bool)
    for j in range(k):
        col = oi[:, j:j + 1]
        present = (gi == col).any(axis=1)
        missing |= must[:, j] & ~present
    fails["missing_neighbour"] = int(missing.sum())

    err = np.abs(gd - delta_g)
    bad = (err > tol_dist * delta_g) | ((delta_g == 0) & (gd != 0))
    fails["distance_error"] = int((bad & in_range).any(axis=1).sum())
    fails["unsorted"] = int((np.diff(gd, axis=1) < 0).any(axis=1).sum()) if k > 1 else 0

    exact_sets = (np.sort(gi, axis=1) == np.sort(oi, axis=1)).all(axis=1)
    info = {
        "rows": len(rows),
        "identical_sets": int(exact_sets.sum()),
        "max_rel_dist_err": float(np.max(np.where(delta_g > 0, err / np.maximum(delta_g, 1e-300), 0))),
    }
    return fails, info


def assert_ok(*args, **kw):
    fails, info = check(*args, **kw)
    bad = {k: v for k, v in fails.items() if v}
    assert not bad, f"parity failures {bad} ({info})"
    return info


def check_furthest(q, r, k, gpu_idx, gpu_dist, ora_idx, ora_d2, rows=None,
                   exclude_self=False, tol_set=TOL_SET, tol_dist=TOL_DIST):
    """The same predicate for k-furthest lists (descending distances):
    {r : delta_r > delta_k (1 + tol_set)} is a subset of G, G is a subset of
    {r : delta_r >= delta_k (1 - tol_set)}, distances within tol_dist of
    FP64 and non-increasing.  Returns (failure counts, info)."""
    q = np.asarray(q, np.float32)
    r = np.asarray(r, np.float32)
    m = r.shape[0]
    rows = np.arange(q.shape[0]) if rows is None else np.asarray(rows, np.int64)
    gi = np.asarray(gpu_idx)[rows].astype(np.int64)
    gd = np.asarray(gpu_dist)[rows].astype(np.float64)
    oi = np.asarray(ora_idx, np.int64)
    od2 = np.asarray(ora_d2, np.float64)
    assert gi.shape == (len(rows), k) and oi.shape == gi.shape

    fails = {}
    in_range = (gi >= 0) & (gi < m)
    fails["out_of_range"] = int((~in_range).sum())
    gi_safe = np.where(in_range, gi, 0)
    srt = np.sort(gi_safe, axis=1)
    fails["duplicates"] = int((srt[:, 1:] == srt[:, :-1]).any(axis=1).sum()) if k > 1 else 0
    fails["self_match"] = int((gi == rows[:, None]).any(axis=1).sum()) if exclude_self else 0
    qi = np.repeat(rows, k)
    delta_g = np.sqrt(_knn.pair_d2(q, r, qi, gi_safe.ravel()).reshape(len(rows), k))
    delta_o = np.sqrt(od2)
    dk = delta_o[:, k - 1:k]
    lower = delta_g >= dk * (1.0 - tol_set)
    fails["beyond_kth"] = int((~lower & in_range).any(axis=1).sum())
    must = delta_o > dk * (1.0 + tol_set)
    missing = np.zeros(len(rows), bool)
    for j in range(k):
        present = (gi == oi[:, j:j + 1]).any(axis=1)
        missing |= must[:, j] & ~present
    fails["missing_neighbour"] = int(missing.sum())
    err = np.abs(gd - delta_g)
    bad = (err > tol_dist * delta_g) | ((delta_g == 0) & (gd != 0))
    fails["distance_error"] = int((bad & in_range).any(axis=1).sum())
    fails["unsorted"] = int((np.diff(gd, axis=1) > 0).any(axis=1).sum()) if k > 1 else 0
    exact_sets = (np.sort(gi, axis=1) == np.sort(oi, axis=1)).all(axis=1)
    return fails, {"rows": len(rows), "identical_sets": int(exact_sets.sum())}


def assert_ok_furthest(*args, **kw):
    fails, info = check_furthest(*args, **kw)
    bad = {a: b for a, b in fails.items() if b}
    assert not bad, f"parity failures {bad} ({info})"
    return info
