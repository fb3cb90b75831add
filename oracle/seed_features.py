"""Seed-network input features computed from the oracle kd-tree (test
infrastructure only).  Definitions, per query leaf:

* centre: fl32(0.5 * fl32(lo + hi)) of the leaf's box (d values);
* lambda: max distance from that centre to the leaf's points;
* count: number of points in the leaf;
* log density: log(count / volume) of the reference leaf reached by
  descending from the root toward the centre, taking at each node the child
  whose box is nearer to the centre (squared box distance with plain FP32
  products and sums; the left child on ties).  Each box extent is clamped
  below at 1e-6 of the root box's extent (+1e-30).

The seed only steers the amount of work (any seed keeps the search exact),
so these definitions are the library's choice, not the paper's.
"""
from __future__ import annotations

import numpy as np


def _box_d2(lo, hi, c):
    s = np.float32(0.0)
    for j in range(len(c)):
        g = max(max(np.float32(lo[j] - c[j]), np.float32(c[j] - hi[j])), np.float32(0.0))
        s = np.float32(s + np.float32(g * g))
    return s


def features(rtree, qtree):
    d = rtree["d"]
    fl_q = qtree["first_leaf"]
    out = []
    for leaf in range(1 << qtree["depth"]):
        node = fl_q + leaf
        cnt = int(qtree["count"][node])
        if cnt:
            c = (np.float32(0.5) * (qtree["lo"][node] + qtree["hi"][node]).astype(np.float32)).astype(np.float32)
        else:
            c = np.zeros(d, np.float32)
        r = 0
        while r < rtree["first_leaf"]:
            a, b = 2 * r + 1, 2 * r + 2
            da = _box_d2(rtree["lo"][a], rtree["hi"][a], c)
            db = _box_d2(rtree["lo"][b], rtree["hi"][b], c)
            r = b if db < da else a
        ext = (rtree["hi"][r] - rtree["lo"][r]).astype(np.float64)
        root = (rtree["hi"][0] - rtree["lo"][0]).astype(np.float64)
        eps = 1e-6 * root + 1e-30
        logvol = float(np.sum(np.log(np.maximum(ext, eps))))
        dens = np.log(max(float(rtree["count"][r]), 1.0)) - logvol
        out.append(np.concatenate([c.astype(np.float64), [qtree["lam"][node], cnt, dens]]))
    return np.array(out)
