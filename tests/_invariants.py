"""Checks of the k-NN Score log against the paper's correctness argument.

Section "k-Nearest Neighbor Search", the argument after Algorithm 3: a
pruning dual-tree traversal returns the exact answer when Score prunes only
node pairs that cannot hold a true neighbour, which the bound B(N_q)
guarantees because it never falls below the largest true k-th distance of
the node's points.  Given a Score log (one record per call: reference node,
kept flag, the wavefront's query leaves and each leaf's B(N_q)^2), the tree
arrays and the oracle's answer, this module checks both halves:

* every logged bound is at least the largest true squared k-th distance of
  its leaf's points (with the kernel's prune slack 2^-16 and the predicate's
  1e-6 tie tolerance);
* no pruned (query leaf group, reference node) pair holds a reference point
  that is strictly inside some query's true k-th distance.
"""
from __future__ import annotations

import numpy as np

SLACK = 1.0 + 2.0 ** -16
TOL = 2e-6


def check_log(log, n_leaves, first_leaf_r, q_start, q_count, q_perm, r_start, r_count, r_perm,
              ora_idx, ora_d2, k):
    """Return (bound_violations, prune_violations, n_pruned).

    log: [n, 12] uint32 records; q_start/q_count: query leaf ranges (leaf
    order, tree positions); r_start/r_count: reference node ranges (heap
    order); q_perm/r_perm: tree position -> original row; ora_idx/ora_d2:
    oracle lists by original query row."""
    log = np.asarray(log, np.uint32)
    node = log[:, 0].astype(np.int64)
    kept = log[:, 1] != 0
    first = log[:, 2].astype(np.int64)
    ng = log[:, 3].astype(np.int64)
    bounds = log[:, 4:12].view(np.float32).astype(np.float64)

    # largest true squared k-th distance per query leaf
    kth = np.asarray(ora_d2, np.float64)[:, k - 1]
    need = np.full(n_leaves, -np.inf)
    for leaf in range(n_leaves):
        s, c = q_start[leaf], q_count[leaf]
        if c:
            need[leaf] = kth[q_perm[s:s + c]].max()
    bound_bad = 0
    for g in range(bounds.shape[1]):
        leaf = first + g
        on = (g < ng) & (leaf < n_leaves)
        nl = need[np.where(on, leaf, 0)]
        bad = on & (bounds[:, g] * SLACK < nl * (1.0 - TOL))
        bound_bad += int(bad.sum())

    # strict true neighbours of every query position, as reference positions
    r_pos = np.empty_like(r_perm)
    r_pos[r_perm] = np.arange(len(r_perm))
    strict = np.asarray(ora_d2, np.float64) < kth[:, None] * (1.0 - TOL)   # by original row
    nb_pos = np.where(strict, r_pos[np.asarray(ora_idx, np.int64)], -1)    # by original row
    nb_by_qpos = nb_pos[q_perm]                                           # by query position
    prune_bad = 0
    pruned = np.nonzero(~kept)[0]
    for i in pruned:
        lo_leaf = first[i]
        hi_leaf = min(first[i] + ng[i], n_leaves)
        qs = q_start[lo_leaf]
        qe = q_start[hi_leaf - 1] + q_count[hi_leaf - 1]
        s, c = r_start[node[i]], r_count[node[i]]
        block = nb_by_qpos[qs:qe]
        prune_bad += int(((block >= s) & (block < s + c)).any())
    return bound_bad, prune_bad, int(len(pruned))
