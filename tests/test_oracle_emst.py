"""Pins of the minimum-spanning-tree oracle (Section "Boruvka's Algorithm"):
Figure 1 with a hand-derived tree, Kruskal in numpy, scipy's spanning tree
on the dense distance matrix, the lattice closed form, the cut property on
small inputs, and the literal dual-tree Boruvka (Algorithms 7 and 8 with the
merge loop) reaching the same tree under every bound."""
import os

import numpy as np
import pytest

from oracle import dualtree as dt
from oracle import knn as ok
from paper_1304_4327_amd import datagen

FIG1 = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)


def test_figure1_tree(golden_dir):
    edges, total = [], None
    for line in open(os.path.join(golden_dir, "fig1_emst.txt")):
        t = line.split("#", 1)[0].split()
        if t and t[0] == "edge":
            edges.append((int(t[1]), int(t[2]), float(t[3])))
        elif t and t[0] == "total":
            total = float(t[1])
    u, v, d2 = ok.emst(FIG1)
    want = np.array([(a, b) for a, b, _ in edges])
    assert np.array_equal(ok.edge_set(u, v), ok.edge_set(want[:, 0], want[:, 1]))
    assert sorted(d2.tolist()) == sorted(w for _, _, w in edges)
    assert abs(np.sqrt(d2).sum() - total) < 1e-15


def test_kruskal_and_scipy_agree():
    from scipy.sparse.csgraph import minimum_spanning_tree
    rng = np.random.default_rng(4)
    for n, d in [(2, 3), (7, 1), (60, 2), (150, 5)]:
        x = rng.random((n, d)).astype(np.float32)
        u, v, d2 = ok.emst(x)
        ku, kv, kd2 = ok.emst_kruskal(x)
        assert np.array_equal(ok.edge_set(u, v), ok.edge_set(ku, kv))
        x64 = x.astype(np.float64)
        dense = np.sqrt(((x64[:, None] - x64[None]) ** 2).sum(-1))
        assert abs(minimum_spanning_tree(dense).sum() - np.sqrt(d2).sum()) < 1e-9


def test_ties_follow_the_total_order():
    """Equal lengths everywhere (a unit lattice): the tree is the one the
    order (length, smaller index, larger index) picks, and its length is
    n - 1."""
    g = datagen.lattice(5, 3)
    u, v, d2 = ok.emst(g)
    ku, kv, _ = ok.emst_kruskal(g)
    assert np.array_equal(ok.edge_set(u, v), ok.edge_set(ku, kv))
    assert np.all(d2 == 1.0) and len(d2) == len(g) - 1


def test_cut_property():
    """Every tree edge is the lightest edge across the cut it defines."""
    rng = np.random.default_rng(9)
    x = rng.random((40, 2)).astype(np.float32)
    u, v, d2 = ok.emst(x)
    x64 = x.astype(np.float64)
    dense = ((x64[:, None] - x64[None]) ** 2).sum(-1)
    for e in range(len(u)):
        adj = {i: set() for i in range(len(x))}
        for f in range(len(u)):
            if f != e:
                adj[u[f]].add(v[f])
                adj[v[f]].add(u[f])
        side, stack = {u[e]}, [u[e]]
        while stack:
            for w in adj[stack.pop()]:
                if w not in side:
                    side.add(w)
                    stack.append(w)
        a = np.array(sorted(side))
        b = np.array(sorted(set(range(len(x))) - side))
        assert dense[np.ix_(a, b)].min() == d2[e]


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
def test_literal_dual_tree_boruvka(bound):
    for seed in range(150):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 60))
        d = int(rng.integers(1, 4))
        x = rng.random((n, d)).astype(np.float32)
        if seed % 3 == 1:
            x[: n // 2] = (0.5 + 0.01 * rng.random((n // 2, d))).astype(np.float32)
        if seed % 3 == 2:
            x = np.round(x * 4).astype(np.float32)      # duplicates and ties
        t = dt.DualTreeBoruvka(x, int(rng.integers(1, 6)), bound)
        u, v, _ = t.run()
        pu, pv, _ = ok.emst(x)
        assert np.array_equal(ok.edge_set(u, v), ok.edge_set(pu, pv)), seed


def test_literal_dual_tree_boruvka_prunes():
    x = datagen.uniform(400, 2, 8)
    tb = dt.DualTreeBoruvka(x, 4, "B")
    tb.run()
    tn = dt.DualTreeBoruvka(x, 4, "none")
    tn.run()
    assert tb.base_cases < 0.5 * tn.base_cases
