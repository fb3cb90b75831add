"""Plain recursive kd-tree build (test infrastructure only).

A kd-tree is a space tree (Definition 1, Section "Space Trees"): every node
owns an axis-aligned box (its convex set) that contains its points and its
children's boxes; points are held only by leaves (Section on Gray's AllNN:
kd-trees hold points only in leaves).  The paper does not fix a split rule;
the build follows this one, written here in the most direct form:

* the tree is complete, of depth L = smallest L >= 0 with ceil(N / 2^L) <=
  leaf_size, nodes numbered in heap order (children of i are 2i+1, 2i+2);
* a node with n points splits on the dimension of largest box extent
  (hi - lo in FP32; ties -> lowest dimension);
* its left child receives the floor(n/2) smallest points under the order
  (coordinate on that dimension, original index), the right child the rest;
* each child keeps its points in ascending original index, and the
  permutation is the concatenation of the leaves' index lists, so every
  node's points occupy a contiguous range of it;
* the box is the tight FP32 min/max of the node's points (empty node:
  lo = +inf, hi = -inf), the centre C = fl32(0.5 * fl32(lo + hi)), and
  lambda = max over the node's points of ||C - p|| (the maximum descendant
  distance of Section "Space Trees"), computed exactly in FP64.  At a kd-tree
  leaf rho = lambda (all of a leaf's descendant points are held points).
"""
from __future__ import annotations

import numpy as np


def depth_for(n: int, leaf_size: int) -> int:
    L = 0
    while -(-n // (1 << L)) > leaf_size:
        L += 1
    return L


def build(points, leaf_size: int):
    pts = np.ascontiguousarray(points, dtype=np.float32)
    n, d = pts.shape
    L = depth_for(n, leaf_size)
    n_nodes = (1 << (L + 1)) - 1
    first_leaf = (1 << L) - 1
    members = [None] * n_nodes
    members[0] = np.arange(n, dtype=np.int64)
    split_dim = np.full(n_nodes, -1, np.int32)
    lo = np.full((n_nodes, d), np.inf, np.float32)
    hi = np.full((n_nodes, d), -np.inf, np.float32)
    for node in range(n_nodes):
        idx = members[node]
        if idx.size:
            lo[node] = pts[idx].min(axis=0)
            hi[node] = pts[idx].max(axis=0)
        if node >= first_leaf:
            continue
        ext = (hi[node] - lo[node]).astype(np.float32) if idx.size else np.zeros(d, np.float32)
        j = int(np.argmax(ext))          # first maximum -> lowest dimension on ties
        split_dim[node] = j
        order = np.lexsort((idx, pts[idx, j]))   # by coordinate, then index
        half = idx.size // 2
        members[2 * node + 1] = np.sort(idx[order[:half]])
        members[2 * node + 2] = np.sort(idx[order[half:]])

    perm = np.concatenate([members[first_leaf + i] for i in range(1 << L)])
    start = np.zeros(n_nodes, np.int64)
    count = np.array([m.size for m in members], np.int64)
    # a node's points occupy a contiguous range of the permutation
    start[0] = 0
    for node in range(first_leaf):
        start[2 * node + 1] = start[node]
        start[2 * node + 2] = start[node] + count[2 * node + 1]

    with np.errstate(invalid="ignore"):      # empty nodes: inf + (-inf)
        centre = (np.float32(0.5) * (lo + hi).astype(np.float32)).astype(np.float32)
    lam = np.zeros(n_nodes, np.float64)
    for node in range(n_nodes):
        idx = members[node]
        if idx.size:
            diff = pts[idx].astype(np.float64) - centre[node].astype(np.float64)
            lam[node] = np.sqrt((diff * diff).sum(axis=1).max())
    return dict(n=n, d=d, leaf_size=leaf_size, depth=L, n_nodes=n_nodes,
                first_leaf=first_leaf, perm=perm, start=start, count=count,
                lo=lo, hi=hi, centre=centre, lam=lam, split_dim=split_dim)


def leaf_of_rows(tree):
    """Query-leaf number (0 .. 2^L - 1) of every original row."""
    out = np.empty(tree["n"], np.int64)
    fl = tree["first_leaf"]
    for i in range(1 << tree["depth"]):
        s, c = tree["start"][fl + i], tree["count"][fl + i]
        out[tree["perm"][s:s + c]] = i
    return out
