"""Literal pruning dual-tree k-NN on tiny inputs (test infrastructure only).

The paper's meta-algorithm (Section "Overview"): a space tree (here the
kd-tree of ``oracle.kdtree``), a pruning dual-tree traversal (Algorithm 1,
depth first), the k-NN BaseCase (Algorithm 2) and the k-NN Score
(Algorithm 3).  Nothing is blocked, fused or reordered; it exists to pin the
reading of the bound B(N_q) and to show that pruning with it is exact.

Traversal detail: Algorithm 1 recurses over C_q x C_r; for a kd-tree, whose
points sit only in leaves, a childless node stands for itself in that
product (the convention of Gray's AllNN, Algorithm 4), and the recursion
stops when both nodes are leaves.  Children of the reference node are taken
closer-first (Algorithm 4).

Bounds (Section "k-Nearest Neighbor Search"):

``B1``      max over the node's descendant points of D_p[k].
``B``       the combined bound, safe reading: the four-way minimum of
            B1(N_q), min_p D_p[k] + rho + lambda (rho = lambda at a kd-tree
            leaf, and every descendant point lies in some leaf, so this is
            min over descendants of D_p[k] + 2 lambda(N_q)), and B(Par(N_q)).
            The printed child term B(N_c) + 2(lambda_q - lambda_c) is left
            out: it is justified only when B(N_c) is attained by its
            minimum-plus-2-lambda term, and the tests exhibit inputs where the
            printed recursion falls below the largest true k-th distance.
``printed`` the recursion exactly as printed, evaluated bottom-up, for
            those tests only.
``none``    never prune (the non-pruning traversal of the correctness
            argument).

Distances are FP64.  Algorithm 3 visits when d_min < B, i.e. prunes when
d_min >= B.  That is safe for B1 (a point at exactly the current k-th
distance is not a strict improvement for the BaseCase) but not for the
minimum-plus-2-lambda term, whose triangle-inequality argument only
guarantees k points at distance <= B, not yet found: with ties (a point at
exactly that distance) the non-strict prune discards a true neighbour.  The
default here is the strict prune d_min > B; ``strict=False`` gives the
printed comparison, for the test that exhibits the difference.
"""
from __future__ import annotations

import math

import numpy as np

from . import kdtree as _kd


class DualTreeKNN:
    def __init__(self, qpts, rpts, k, leaf_size=2, bound="B", exclude_self=False,
                 strict=True):
        self.q = np.asarray(qpts, np.float32).astype(np.float64)
        self.r = np.asarray(rpts, np.float32).astype(np.float64)
        self.k = k
        self.bound = bound
        self.exclude_self = exclude_self
        self.strict = strict
        self.tq = _kd.build(qpts, leaf_size)
        self.tr = _kd.build(rpts, leaf_size)
        n = self.q.shape[0]
        self.D = np.full((n, k), np.inf)       # candidate distances, ascending
        self.N = np.full((n, k), -1, np.int64)  # candidate indices
        self.base_cases = 0
        self.score_calls = 0
        self.visited = set()

    # --- tree helpers -------------------------------------------------------
    def _is_leaf(self, t, node):
        return node >= t["first_leaf"]

    def _children(self, t, node):
        return [] if self._is_leaf(t, node) else [2 * node + 1, 2 * node + 2]

    def _points(self, t, node):
        s, c = t["start"][node], t["count"][node]
        return t["perm"][s:s + c]

    def _held(self, t, node):
        return self._points(t, node) if self._is_leaf(t, node) else np.empty(0, np.int64)

    def _dmin(self, nq, nr):
        """Lower bound on d_min: distance between the two boxes."""
        tq, tr = self.tq, self.tr
        if tq["count"][nq] == 0 or tr["count"][nr] == 0:
            return math.inf
        lo_q, hi_q = tq["lo"][nq].astype(np.float64), tq["hi"][nq].astype(np.float64)
        lo_r, hi_r = tr["lo"][nr].astype(np.float64), tr["hi"][nr].astype(np.float64)
        gap = np.maximum(0.0, np.maximum(lo_r - hi_q, lo_q - hi_r))
        return float(np.sqrt((gap * gap).sum()))

    # --- bounds -------------------------------------------------------------
    def _kth(self, node):
        return self.D[self._points(self.tq, node), self.k - 1]

    def _B_safe(self, node, with_b2=True):
        pts = self._kth(node)
        if pts.size == 0:
            return math.inf
        b = pts.max()
        if with_b2:
            b = min(b, pts.min() + 2.0 * self.tq["lam"][node])
        if node > 0:
            b = min(b, self._B_safe((node - 1) // 2, with_b2))
        return b

    def _B_printed_up(self, node):
        t = self.tq
        if t["count"][node] == 0:
            return math.inf
        held = self.D[self._held(t, node), self.k - 1]
        kids = [c for c in self._children(t, node) if t["count"][c] > 0]
        kb = [self._B_printed_up(c) for c in kids]
        lam = t["lam"][node]
        rho = lam if self._is_leaf(t, node) else 0.0
        maxes = ([held.max()] if held.size else []) + kb
        terms = [max(maxes)]
        if held.size:
            terms.append(held.min() + rho + lam)
        for c, b in zip(kids, kb):
            terms.append(b + 2.0 * (lam - t["lam"][c]))
        return min(terms)

    def _B_printed(self, node):
        b = self._B_printed_up(node)
        if node > 0:
            b = min(b, self._B_printed((node - 1) // 2))
        return b

    def bound_of(self, node):
        if self.bound == "none":
            return math.inf
        if self.bound == "B1":
            return self._B_safe(node, with_b2=False)
        if self.bound == "B":
            return self._B_safe(node, with_b2=True)
        if self.bound == "printed":
            return self._B_printed(node)
        raise ValueError(self.bound)

    # --- the three callbacks ------------------------------------------------
    def score(self, nq, nr):
        self.score_calls += 1
        dmin = self._dmin(nq, nr)
        b = self.bound_of(nq)
        keep = dmin <= b if self.strict else dmin < b
        return dmin if keep else math.inf

    def base_case(self, iq, ir):
        if self.exclude_self and iq == ir:
            return math.inf
        self.base_cases += 1
        diff = self.q[iq] - self.r[ir]
        d = math.sqrt(float(diff @ diff))
        if d < self.D[iq, self.k - 1] and (iq, ir) not in self.visited:
            self.visited.add((iq, ir))
            row_d, row_n = self.D[iq], self.N[iq]
            pos = int(np.searchsorted(row_d, d, side="right"))
            row_d[pos + 1:] = row_d[pos:-1].copy()
            row_n[pos + 1:] = row_n[pos:-1].copy()
            row_d[pos], row_n[pos] = d, ir
        return d

    def traverse(self, nq=0, nr=0):
        if self.score(nq, nr) == math.inf:
            return
        for iq in self._held(self.tq, nq):
            for ir in self._held(self.tr, nr):
                self.base_case(int(iq), int(ir))
        cq = self._children(self.tq, nq) or [nq]
        cr = self._children(self.tr, nr) or [nr]
        if cq == [nq] and cr == [nr]:
            return
        for c in cq:
            # closer reference child first
            order = sorted(cr, key=lambda x: self._dmin(c, x))
            for x in order:
                self.traverse(c, x)

    def run(self):
        self.traverse(0, 0)
        return self.N.copy(), self.D.copy()


def printed_bound_bottom_up(tree, kth):
    """The printed recursion for B(N) (without the parent term) evaluated
    bottom-up from per-point k-th distances ``kth`` (indexed by original
    row), together with the safe-reading value and the true requirement
    max over descendants of kth, for every node."""
    n_nodes, fl = tree["n_nodes"], tree["first_leaf"]
    lam = tree["lam"]
    printed = np.full(n_nodes, np.inf)
    safe = np.full(n_nodes, np.inf)
    need = np.full(n_nodes, -np.inf)
    for node in range(n_nodes - 1, -1, -1):
        s, c = tree["start"][node], tree["count"][node]
        pts = kth[tree["perm"][s:s + c]]
        if pts.size == 0:
            continue
        need[node] = pts.max()
        safe[node] = min(pts.max(), pts.min() + 2.0 * lam[node])
        if node >= fl:
            printed[node] = min(pts.max(), pts.min() + 2.0 * lam[node])
        else:
            kids = [2 * node + 1, 2 * node + 2]
            kb = [printed[x] for x in kids if tree["count"][x] > 0]
            terms = [max(kb)] + [printed[x] + 2.0 * (lam[node] - lam[x])
                                 for x in kids if tree["count"][x] > 0]
            printed[node] = min(terms)
    return printed, safe, need


class DualTreeKFN(DualTreeKNN):
    """Literal k-furthest-neighbour dual-tree search (the closing remark of
    Section "k-Nearest Neighbor Search"): the k-NN rules with max and min
    exchanged, lists kept in descending distance, D initialised to 0 and the
    BaseCase comparison d > D[k].

    Inverted bound (safe reading, the mirror of the k-NN one): every point
    p of N_q ends with a k-th furthest distance of at least
      L1 = min over the node's points of D_p[k]  (the list only grows), and
      L2 = max over the node's points of D_p[k] - 2 lambda(N_q) (the k points
           found for that point are, by the triangle inequality, at least
           that far from every point of the node), and the parent's L,
    so L(N_q) = max{L1, L2, L(Par)}, and a pair whose largest possible
    distance d_max(N_q, N_r) is below L cannot change any list: Score prunes
    iff d_max < L.  ``bound`` is "B" (all three terms), "B1" (L1 and the
    parent) or "none"."""

    def __init__(self, qpts, rpts, k, leaf_size=2, bound="B", exclude_self=False):
        super().__init__(qpts, rpts, k, leaf_size, bound, exclude_self)
        self.D = np.zeros_like(self.D)          # initialised to 0

    def _dmax(self, nq, nr):
        tq, tr = self.tq, self.tr
        if tq["count"][nq] == 0 or tr["count"][nr] == 0:
            return -math.inf
        lo_q, hi_q = tq["lo"][nq].astype(np.float64), tq["hi"][nq].astype(np.float64)
        lo_r, hi_r = tr["lo"][nr].astype(np.float64), tr["hi"][nr].astype(np.float64)
        span = np.maximum(hi_r - lo_q, hi_q - lo_r)
        return float(np.sqrt((span * span).sum()))

    def _L(self, node):
        pts = self._kth(node)
        if pts.size == 0:
            return -math.inf
        b = pts.min()
        if self.bound == "B":
            b = max(b, pts.max() - 2.0 * self.tq["lam"][node])
        if node > 0:
            b = max(b, self._L((node - 1) // 2))
        return b

    def score(self, nq, nr):
        self.score_calls += 1
        dmax = self._dmax(nq, nr)
        if self.bound != "none" and dmax < self._L(nq):
            return math.inf
        return -dmax                         # larger d_max visited first

    def base_case(self, iq, ir):
        if self.exclude_self and iq == ir:
            return 0.0
        self.base_cases += 1
        diff = self.q[iq] - self.r[ir]
        d = math.sqrt(float(diff @ diff))
        if d > self.D[iq, self.k - 1] and (iq, ir) not in self.visited:
            self.visited.add((iq, ir))
            row_d, row_n = self.D[iq], self.N[iq]
            pos = int(np.searchsorted(-row_d, -d, side="right"))
            row_d[pos + 1:] = row_d[pos:-1].copy()
            row_n[pos + 1:] = row_n[pos:-1].copy()
            row_d[pos], row_n[pos] = d, ir
        return d

    def traverse(self, nq=0, nr=0):
        if self.score(nq, nr) == math.inf:
            return
        for iq in self._held(self.tq, nq):
            for ir in self._held(self.tr, nr):
                self.base_case(int(iq), int(ir))
        cq = self._children(self.tq, nq) or [nq]
        cr = self._children(self.tr, nr) or [nr]
        if cq == [nq] and cr == [nr]:
            return
        for c in cq:
            # farther reference child first
            order = sorted(cr, key=lambda x: -self._dmax(c, x))
            for x in order:
                self.traverse(c, x)


class DualTreeRange(DualTreeKNN):
    """Literal range search (Section "Range Search", Algorithms 5 and 6): the
    BaseCase adds every reference whose distance lies in [lo, hi]; Score
    keeps a node pair while some of its pairs may lie in the range.

    Score reading.  As printed, Algorithm 6 keeps a pair only when
    lo <= d_min(N_q, N_r) <= hi, which also discards a pair whose d_min is
    below lo although its farther points lie inside the range (for instance
    any pair of overlapping nodes when lo > 0).  The safe reading keeps the
    pair unless every distance misses the range: prune iff d_min > hi or
    d_max < lo.  ``printed=True`` uses the printed test, for the test that
    shows the difference."""

    def __init__(self, qpts, rpts, lo, hi, leaf_size=2, exclude_self=False, printed=False):
        super().__init__(qpts, rpts, 1, leaf_size, "none", exclude_self)
        self.lo, self.hi, self.printed = lo, hi, printed
        self.found = [set() for _ in range(self.q.shape[0])]

    def score(self, nq, nr):
        self.score_calls += 1
        dmin = self._dmin(nq, nr)
        if self.printed:
            return dmin if self.lo <= dmin <= self.hi else math.inf
        dmax = DualTreeKFN._dmax(self, nq, nr)
        return math.inf if (dmin > self.hi or dmax < self.lo) else dmin

    def base_case(self, iq, ir):
        if self.exclude_self and iq == ir:
            return 0.0
        self.base_cases += 1
        diff = self.q[iq] - self.r[ir]
        s = float(diff @ diff)
        if self.lo * self.lo <= s <= self.hi * self.hi:
            self.found[iq].add(ir)
        return math.sqrt(s)

    def run(self):
        self.traverse(0, 0)
        return [np.array(sorted(f), np.int64) for f in self.found]


class DualTreeKDE(DualTreeKNN):
    """Literal kernel density estimation (Section "Kernel Density
    Estimation", Algorithms 9 and 10) with K(d) = exp(-d^2 / (2 h^2)).

    Score computes B_K = K(d_min) - K(d_max) for the node pair; when it is
    below eps / |S_r| every descendant query point receives
    |D^p_r| K(||p_q - C_r||) with C_r the reference node's centre (the box
    centre, a point of the node's box, so each pair's error is at most B_K)
    and the pair is pruned; otherwise the traversal descends, and BaseCase
    adds K(||p_q - p_r||).  Then |f - exact| <= eps for every query.

    Reading: Algorithm 9 as printed approximates when B_K >= eps / |S_r|,
    the opposite of the text around it (approximate when B_K is below the
    threshold, which is what bounds the error); ``printed=True`` uses the
    printed comparison, for the test that shows its error exceeding eps."""

    def __init__(self, qpts, rpts, h, eps, leaf_size=2, exclude_self=False, printed=False):
        super().__init__(qpts, rpts, 1, leaf_size, "none", exclude_self)
        self.h, self.eps, self.printed = h, eps, printed
        self.f = np.zeros(self.q.shape[0])
        self.approximations = 0

    def _K(self, d):
        return math.exp(-d * d / (2.0 * self.h * self.h))

    def score(self, nq, nr):
        self.score_calls += 1
        dmin = self._dmin(nq, nr)
        if dmin == math.inf:
            return math.inf
        dmax = DualTreeKFN._dmax(self, nq, nr)
        bk = self._K(dmin) - self._K(dmax)
        thr = self.eps / self.r.shape[0]
        approx = bk >= thr if self.printed else bk < thr
        if approx:
            self.approximations += 1
            c = self.tr["centre"][nr].astype(np.float64)
            cnt = self.tr["count"][nr]
            for p in self._points(self.tq, nq):
                diff = self.q[p] - c
                self.f[p] += cnt * self._K(math.sqrt(float(diff @ diff)))
            return math.inf
        return dmin

    def base_case(self, iq, ir):
        if self.exclude_self and iq == ir:
            return 0.0
        self.base_cases += 1
        diff = self.q[iq] - self.r[ir]
        d = math.sqrt(float(diff @ diff))
        self.f[iq] += self._K(d)
        return d

    def run(self):
        self.traverse(0, 0)
        return self.f.copy()


class DualTreeBoruvka(DualTreeKNN):
    """Literal dual-tree Boruvka (Section "Boruvka's Algorithm", Algorithms 7
    and 8 and the traversal-merge loop) on one kd-tree used as both trees.

    Per round, for every component F_i: D(F_i), N(F_i), p_c(F_i).  BaseCase
    (Algorithm 7) offers the pair (p_q, p_r) to F(p_q) when the two lie in
    different components; Score (Algorithm 8) prunes a node pair whose points
    all lie in one component, or whose d_min exceeds B(N_q).  After the
    traversal each component's edge (p_c, N) is added and components joined
    by an edge are merged, until one remains.

    Readings.
    * Ties: the BaseCase comparison "d < D(F(p_q))" keeps the first of equal
      distances, which depends on visit order and, with equal-length edges,
      can close a cycle; candidates are compared by the strict total order
      (squared length, smaller index, larger index) instead, under which the
      minimum spanning tree is unique and Boruvka's merges never form a
      cycle.  The prune is strict (d_min > B), so a tie is never pruned.
    * The bound is Section 5's B(N_q) with k = 1 and D_p[1] = D(F(p)) (the
      safe reading, without the printed child term): B1 = max_p D(F(p)),
      B2 = min_p D(F(p)) + 2 lambda(N_q), and the parent's.  B2 stays a
      bound although D(F(p)) is realised elsewhere in the component: if the
      node holds points of two components, each of them has an edge of
      length at most 2 lambda (between those two points), so its shortest
      edge is at most B2; if it holds one component c, B2 >= D(c) = B1.
      ``bound`` is "B" (all terms), "B1" (max term and parent) or "none"
      (prune only node pairs inside one component)."""

    def __init__(self, pts, leaf_size=2, bound="B"):
        super().__init__(pts, pts, 1, leaf_size, "none", False)
        self.mode = bound
        n = self.q.shape[0]
        self.F = np.arange(n)
        self.edges = []
        self.rounds = 0

    def _same_component(self, nq, nr):
        a = self.F[self._points(self.tq, nq)]
        b = self.F[self._points(self.tr, nr)]
        return a.size == 0 or b.size == 0 or (np.all(a == a[0]) and np.all(b == a[0]))

    def _B(self, node):
        if self.mode == "none":
            return math.inf
        pts = self._points(self.tq, node)
        if pts.size == 0:
            return math.inf
        dk = np.array([self.D[self.F[p]] for p in pts])
        b = dk.max()
        if self.mode == "B":
            b = min(b, dk.min() + 2.0 * self.tq["lam"][node])
        if node > 0:
            b = min(b, self._B((node - 1) // 2))
        return b

    def score(self, nq, nr):
        self.score_calls += 1
        if self._same_component(nq, nr):
            return math.inf
        dmin = self._dmin(nq, nr)
        return math.inf if dmin > self._B(nq) else dmin

    def base_case(self, iq, ir):
        if iq == ir:
            return 0.0
        self.base_cases += 1
        diff = self.q[iq] - self.q[ir]
        s = float(diff @ diff)
        c = self.F[iq]
        if self.F[ir] != c:
            key = (s, min(iq, ir), max(iq, ir))
            if self.best[c] is None or key < self.best[c]:
                self.best[c] = key
                self.D[c] = math.sqrt(s)
        return math.sqrt(s)

    def run(self):
        n = self.q.shape[0]
        while len(set(self.F.tolist())) > 1:
            self.rounds += 1
            self.D = np.full(n, math.inf)     # indexed by component label
            self.best = [None] * n
            self.traverse(0, 0)
            # merge: every component's edge, once
            chosen = {self.best[c] for c in set(self.F.tolist()) if self.best[c] is not None}
            parent = list(range(n))

            def root(a):
                while parent[a] != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a

            for (s, a, b) in sorted(chosen):
                ra, rb = root(self.F[a]), root(self.F[b])
                if ra == rb:
                    raise RuntimeError("a chosen edge closes a cycle")
                parent[ra] = rb
                self.edges.append((a, b, s))
            self.F = np.array([root(self.F[i]) for i in range(n)])
            if not chosen:
                raise RuntimeError("no edge found while several components remain")
        if not self.edges:
            return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
        u, v, w = zip(*self.edges)
        return np.array(u, np.int64), np.array(v, np.int64), np.array(w)
