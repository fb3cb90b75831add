"""FP64 brute-force k-NN oracle (test infrastructure only).

``knn(q, r, k, exclude_self)`` is the definition the dual-tree method reaches
exactly (Section "k-Nearest Neighbor Search": the problem statement -- for
each query the k nearest references and their distances, 0 < k < m -- and the
brute-force remark that every pair is compared and the k smallest kept).  The
work runs in ``knn_bruteforce.c`` (OpenMP); ``knn_numpy`` is the same
definition in a few lines of numpy for tiny inputs.

Ties are ordered by reference index; with ``exclude_self`` (query set equal to
the reference set, the footnote to the k-NN BaseCase) reference i is skipped
for query i by index identity.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        p = ctypes.c_void_p
        lib.knn_oracle_bruteforce.argtypes = [p, i64, p, i64, i32, i32, i32, p, p]
        lib.knn_oracle_bruteforce.restype = ctypes.c_int
        lib.knn_oracle_bruteforce_rows.argtypes = [p, p, i64, p, i64, i32, i32, i32, p, p]
        lib.knn_oracle_bruteforce_rows.restype = ctypes.c_int
        lib.knn_oracle_pair_d2.argtypes = [p, p, i32, p, p, i64, p]
        lib.knn_oracle_pair_d2.restype = ctypes.c_int
        lib.knn_oracle_threads.restype = ctypes.c_int
        lib.knn_oracle_furthest_rows.argtypes = [p, p, i64, p, i64, i32, i32, i32, p, p]
        lib.knn_oracle_furthest_rows.restype = ctypes.c_int
        lib.knn_oracle_range_rows.argtypes = [p, p, i64, p, i64, i32, ctypes.c_double,
                                              ctypes.c_double, i32, p, p, p, p]
        lib.knn_oracle_range_rows.restype = ctypes.c_int
        lib.knn_oracle_kde_rows.argtypes = [p, p, i64, p, i64, i32, ctypes.c_double, i32, p, p]
        lib.knn_oracle_kde_rows.restype = ctypes.c_int
        lib.knn_oracle_emst.argtypes = [p, i64, i32, p, p, p]
        lib.knn_oracle_emst.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def threads() -> int:
    return int(_load().knn_oracle_threads())


def knn(q, r, k: int, exclude_self: bool = False):
    """All queries.  Returns (idx int64 [n,k], d2 float64 [n,k])."""
    q, r = _f32(q), _f32(r)
    n, d = q.shape
    m = r.shape[0]
    idx = np.empty((n, k), np.int64)
    d2 = np.empty((n, k), np.float64)
    rc = _load().knn_oracle_bruteforce(q.ctypes.data, n, r.ctypes.data, m, d, k,
                                       int(bool(exclude_self)), idx.ctypes.data,
                                       d2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments (need 0 < k < m)")
    return idx, d2


def knn_rows(q, rows, r, k: int, exclude_self: bool = False):
    """Queries ``q[rows]`` only (rows are indices into q)."""
    q, r = _f32(q), _f32(r)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    d = q.shape[1]
    m = r.shape[0]
    idx = np.empty((len(rows), k), np.int64)
    d2 = np.empty((len(rows), k), np.float64)
    rc = _load().knn_oracle_bruteforce_rows(q.ctypes.data, rows.ctypes.data, len(rows),
                                            r.ctypes.data, m, d, k,
                                            int(bool(exclude_self)), idx.ctypes.data,
                                            d2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments (need 0 < k < m)")
    return idx, d2


def pair_d2(q, r, qi, ri):
    """FP64 squared distance of explicit pairs (q[qi[t]], r[ri[t]])."""
    q, r = _f32(q), _f32(r)
    qi = np.ascontiguousarray(qi, dtype=np.int64).ravel()
    ri = np.ascontiguousarray(ri, dtype=np.int64).ravel()
    out = np.empty(qi.shape[0], np.float64)
    rc = _load().knn_oracle_pair_d2(q.ctypes.data, r.ctypes.data, q.shape[1],
                                    qi.ctypes.data, ri.ctypes.data, qi.shape[0],
                                    out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return out


def knn_numpy(q, r, k: int, exclude_self: bool = False):
    """The same definition in numpy (tiny inputs): full distance matrix, then
    a stable sort on (distance, index)."""
    q = np.asarray(q, np.float32).astype(np.float64)
    r = np.asarray(r, np.float32).astype(np.float64)
    diff = q[:, None, :] - r[None, :, :]
    d2 = np.einsum("ijk,ijk->ij", diff, diff)
    if exclude_self:
        np.fill_diagonal(d2, np.inf)
    order = np.argsort(d2, axis=1, kind="stable")[:, :k]
    return order.astype(np.int64), np.take_along_axis(d2, order, axis=1)


# --------------------------------------------------------------------------
# k-furthest neighbours (closing remark of Section "k-Nearest Neighbor
# Search"): the k references at the largest distances, descending; equal
# distances by reference index.
# --------------------------------------------------------------------------
def furthest_rows(q, rows, r, k: int, exclude_self: bool = False):
    """Queries ``q[rows]`` only.  Returns (idx int64 [len(rows), k], d2
    float64), distances descending."""
    q, r = _f32(q), _f32(r)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    idx = np.empty((len(rows), k), np.int64)
    d2 = np.empty((len(rows), k), np.float64)
    rc = _load().knn_oracle_furthest_rows(q.ctypes.data, rows.ctypes.data, len(rows),
                                          r.ctypes.data, r.shape[0], q.shape[1], k,
                                          int(bool(exclude_self)), idx.ctypes.data,
                                          d2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments (need 0 < k < m)")
    return idx, d2


def furthest(q, r, k: int, exclude_self: bool = False):
    return furthest_rows(q, np.arange(len(q)), r, k, exclude_self)


def furthest_numpy(q, r, k: int, exclude_self: bool = False):
    """The same definition in numpy (tiny inputs): a stable sort on
    (-distance, index)."""
    q = np.asarray(q, np.float32).astype(np.float64)
    r = np.asarray(r, np.float32).astype(np.float64)
    diff = q[:, None, :] - r[None, :, :]
    d2 = np.einsum("ijk,ijk->ij", diff, diff)
    if exclude_self:
        np.fill_diagonal(d2, -np.inf)
    order = np.argsort(-d2, axis=1, kind="stable")[:, :k]
    return order.astype(np.int64), np.take_along_axis(d2, order, axis=1)


# --------------------------------------------------------------------------
# Range search (Section "Range Search"): every reference at a distance in
# [lo, hi], decided on FP64 squared distances (lo^2 <= s <= hi^2).
# --------------------------------------------------------------------------
def range_rows(q, rows, r, lo: float, hi: float, exclude_self: bool = False):
    """Queries ``q[rows]``.  Returns (offsets int64 [len(rows)+1], idx int64,
    d2 float64): the neighbours of row t are idx[offsets[t]:offsets[t+1]] in
    increasing reference index."""
    q, r = _f32(q), _f32(r)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = len(rows)
    counts = np.empty(n, np.int64)
    lib = _load()
    rc = lib.knn_oracle_range_rows(q.ctypes.data, rows.ctypes.data, n, r.ctypes.data,
                                   r.shape[0], q.shape[1], float(lo), float(hi),
                                   int(bool(exclude_self)), counts.ctypes.data, None, None, None)
    if rc != 0:
        raise ValueError("oracle: invalid arguments (need 0 <= lo <= hi)")
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.empty(offsets[-1], np.int64)
    d2 = np.empty(offsets[-1], np.float64)
    lib.knn_oracle_range_rows(q.ctypes.data, rows.ctypes.data, n, r.ctypes.data, r.shape[0],
                              q.shape[1], float(lo), float(hi), int(bool(exclude_self)),
                              counts.ctypes.data, offsets.ctypes.data, idx.ctypes.data,
                              d2.ctypes.data)
    return offsets, idx, d2


def range_search(q, r, lo: float, hi: float, exclude_self: bool = False):
    return range_rows(q, np.arange(len(q)), r, lo, hi, exclude_self)


def range_numpy(q, r, lo: float, hi: float, exclude_self: bool = False):
    """The same definition in numpy (tiny inputs): a list of index arrays."""
    q = np.asarray(q, np.float32).astype(np.float64)
    r = np.asarray(r, np.float32).astype(np.float64)
    out = []
    for i in range(len(q)):
        diff = r - q[i]
        s = (diff * diff).sum(1)
        keep = (s >= lo * lo) & (s <= hi * hi)
        if exclude_self:
            keep[i] = False
        out.append(np.nonzero(keep)[0])
    return out


# --------------------------------------------------------------------------
# Kernel density sums (Section "Kernel Density Estimation"): f(q) = sum over
# references of exp(-||q - r||^2 / (2 h^2)), FP64.
# --------------------------------------------------------------------------
def kde_rows(q, rows, r, h: float, exclude_self: bool = False):
    """Queries ``q[rows]``.  Returns (f, budget) float64: the exact sums and
    sum K (1 + d^2 / 2h^2), the scale of FP32 evaluation error."""
    q, r = _f32(q), _f32(r)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    f = np.empty(len(rows), np.float64)
    b = np.empty(len(rows), np.float64)
    rc = _load().knn_oracle_kde_rows(q.ctypes.data, rows.ctypes.data, len(rows), r.ctypes.data,
                                     r.shape[0], q.shape[1], float(h), int(bool(exclude_self)),
                                     f.ctypes.data, b.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments (need h > 0)")
    return f, b


def kde(q, r, h: float, exclude_self: bool = False):
    return kde_rows(q, np.arange(len(q)), r, h, exclude_self)


def kde_numpy(q, r, h: float, exclude_self: bool = False):
    q = np.asarray(q, np.float32).astype(np.float64)
    r = np.asarray(r, np.float32).astype(np.float64)
    diff = q[:, None, :] - r[None, :, :]
    k = np.exp(-(diff * diff).sum(-1) / (2.0 * h * h))
    if exclude_self:
        np.fill_diagonal(k, 0.0)
    return k.sum(1)


# --------------------------------------------------------------------------
# Euclidean minimum spanning tree (Section "Boruvka's Algorithm"): unique
# under the edge order (squared length, smaller index, larger index).
# --------------------------------------------------------------------------
def emst(x):
    """Prim's algorithm in FP64 (C).  Returns (u int64 [n-1], v int64, d2
    float64) with u < v, in the order Prim adds the edges."""
    x = _f32(x)
    n = x.shape[0]
    u = np.empty(max(n - 1, 0), np.int64)
    v = np.empty(max(n - 1, 0), np.int64)
    d2 = np.empty(max(n - 1, 0), np.float64)
    rc = _load().knn_oracle_emst(x.ctypes.data, n, x.shape[1], u.ctypes.data, v.ctypes.data,
                                 d2.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return u, v, d2


def emst_kruskal(x):
    """Kruskal's algorithm in numpy (tiny inputs): every edge sorted by
    (squared length, smaller index, larger index), union-find."""
    x = np.asarray(x, np.float32).astype(np.float64)
    n = len(x)
    iu, iv = np.triu_indices(n, 1)
    diff = x[iu] - x[iv]
    d2 = (diff * diff).sum(1)
    order = np.lexsort((iv, iu, d2))
    parent = list(range(n))

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    out = []
    for e in order:
        a, b = root(iu[e]), root(iv[e])
        if a != b:
            parent[a] = b
            out.append((iu[e], iv[e], d2[e]))
    if not out:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    u, v, w = zip(*out)
    return np.array(u, np.int64), np.array(v, np.int64), np.array(w)


def edge_set(u, v):
    """Canonical form of an edge list: sorted (min, max) pairs."""
    a, b = np.minimum(u, v), np.maximum(u, v)
    o = np.lexsort((b, a))
    return np.stack([a[o], b[o]], 1)
