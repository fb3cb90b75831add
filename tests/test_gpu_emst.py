"""Euclidean minimum spanning tree on the GPU (knn_emst, dual-tree Boruvka,
Section "Boruvka's Algorithm") against the FP64 oracle.  Under the edge
order (FP64 squared length, smaller index, larger index) the tree is
unique, so the edge sets must be identical, and each reported length is
FP32 of the FP64 length.  At 1M points, where Prim's O(n^2) is out of
reach, the properties that hold at any size are checked: n - 1 edges that
span, exact lengths, and the cut property on sampled edges."""
import numpy as np
import pytest

from oracle import knn as ok
from paper_1304_4327_amd import datagen

pytestmark = pytest.mark.gpu

FIG1 = np.array([[2, 2], [1, 2.5], [0.5, 0.5], [1, 3], [1.5, 2.5]], np.float32)


def _emst(x, leaf, bound="B", stats=False):
    import torch
    from paper_1304_4327_amd import knn
    t = knn.knn_build_tree(torch.from_numpy(x).cuda(), leaf)
    u, v, w, rounds, st = knn.knn_emst(t, bound=bound, stats=stats)
    torch.cuda.synchronize()
    t.close()
    return u.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy(), rounds, st


def _lengths_exact(x, u, v, w):
    d2 = ok.pair_d2(x, x, u, v)
    np.testing.assert_array_equal(w, np.sqrt(d2).astype(np.float32))


def _check(x, got):
    u, v, w = got[:3]
    assert np.all(u < v)
    pu, pv, _ = ok.emst(x)
    assert np.array_equal(ok.edge_set(u, v), ok.edge_set(pu, pv))
    _lengths_exact(x, u, v, w)


@pytest.mark.parametrize("leaf", [1, 2, 5])
def test_figure1(leaf):
    got = _emst(FIG1, leaf)
    _check(FIG1, got)
    assert abs(float(np.sqrt(ok.pair_d2(FIG1, FIG1, got[0], got[1])).sum())
               - 3.7686595939953778) < 1e-12


@pytest.mark.parametrize("bound", ["B", "B1", "none"])
def test_small_sets_ties_and_duplicates(bound):
    rng = np.random.default_rng(11)
    for trial in range(12):
        n = int(rng.integers(2, 400))
        d = int(rng.integers(1, 9))
        x = rng.random((n, d)).astype(np.float32)
        if trial % 3 == 1:
            x = np.round(x * 3).astype(np.float32)        # many ties, duplicates
        if trial % 3 == 2:
            x[: n // 2] = x[0]                            # a block of duplicates
        _check(x, _emst(x, int(rng.integers(1, 33)), bound))


def test_lattice_all_ties():
    g = datagen.lattice(10, 3)
    got = _emst(g, 8)
    _check(g, got)
    assert np.all(got[2] == 1.0)


@pytest.mark.parametrize("name,scale", [("uniform10k_d3_k5", 1.0), ("gmm1m_d3_k10", 0.02),
                                        ("zipfgmm2m_d8_k10", 0.005),
                                        ("manifold4m_d16_k10", 0.0025),
                                        ("manifold1m_d64_k50", 0.005)])
def test_workload_shapes(name, scale):
    ref, _, _, leaf = datagen.make(name, scale=scale)
    got = _emst(ref, leaf, stats=True)
    _check(ref, got)
    print(f"{name} n={len(ref)}: {got[3]} rounds, {got[4]['pairs'] / len(ref):.0f} pairs/point",
          flush=True)


def test_100k_against_prim():
    ref, _, _, leaf = datagen.make("gmm1m_d3_k10", scale=0.1)
    got = _emst(ref, leaf, stats=True)
    _check(ref, got)
    print(f"100k: {got[3]} rounds, {got[4]['ms_search']:.2f} ms", flush=True)


def _spans(n, u, v):
    parent = np.arange(n)

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in zip(u.tolist(), v.tolist()):
        ra, rb = root(a), root(b)
        if ra == rb:
            return False
        parent[ra] = rb
    return True


def _small_sides(n, u, v, limit, count, seed):
    """Tree edges whose removal cuts off at most `limit` points: (edge index,
    the small side's points)."""
    adj = [[] for _ in range(n)]
    for e, (a, b) in enumerate(zip(u.tolist(), v.tolist())):
        adj[a].append((b, e))
        adj[b].append((a, e))
    # iterative DFS from 0: parent edge and subtree of every vertex
    order, par, pedge = [0], np.full(n, -1), np.full(n, -1)
    seen = np.zeros(n, bool)
    seen[0] = True
    i = 0
    while i < len(order):
        a = order[i]
        i += 1
        for b, e in adj[a]:
            if not seen[b]:
                seen[b] = True
                par[b], pedge[b] = a, e
                order.append(b)
    size = np.ones(n, np.int64)
    for a in reversed(order[1:]):
        size[par[a]] += size[a]
    cand = [a for a in order[1:] if size[a] <= limit]
    rng = np.random.default_rng(seed)
    picks = rng.choice(len(cand), size=min(count, len(cand)), replace=False)
    out = []
    for p in picks:
        top = cand[p]
        side, stack = [top], [top]
        while stack:
            a = stack.pop()
            for b, _ in adj[a]:
                if b != par[a] and par[b] == a:
                    side.append(b)
                    stack.append(b)
        out.append((int(pedge[top]), np.array(side)))
    return out


def test_full_size_properties():
    """1M points (d = 3 Gaussian mixture): n - 1 edges that span, lengths
    exact, and the cut property on 64 sampled edges whose small side has at
    most 50 points -- the edge is the lightest (in the edge order) between
    the side and the rest, found with the oracle's k-NN of the side's
    points."""
    ref, _, _, leaf = datagen.make("gmm1m_d3_k10")
    n = len(ref)
    u, v, w, rounds, st = _emst(ref, leaf, stats=True)
    print(f"emst 1M: {rounds} rounds, {st['ms_search']:.1f} ms, "
          f"{st['pairs'] / n:.0f} pairs/point", flush=True)
    assert len(u) == n - 1 and np.all(u < v)
    assert _spans(n, u, v)
    sample = np.random.default_rng(3).choice(n - 1, 4096, replace=False)
    _lengths_exact(ref, u[sample], v[sample], w[sample])
    for e, side in _small_sides(n, u, v, 50, 64, seed=5):
        k = len(side) + 1
        oi, od2 = ok.knn_rows(ref, side, ref, k)
        inside = np.isin(oi, side)
        best = None
        for row, a in enumerate(side):
            j = int(np.argmax(~inside[row]))          # nearest point outside the side
            key = (od2[row, j], min(a, oi[row, j]), max(a, oi[row, j]))
            best = key if best is None or key < best else best
        want = (float(ok.pair_d2(ref, ref, [u[e]], [v[e]])[0]), int(u[e]), int(v[e]))
        assert best == want, (e, best, want)
