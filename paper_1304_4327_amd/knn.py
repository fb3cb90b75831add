"""ctypes binding of ``libknn_dualtree.so`` (C ABI in ``include/knn.h``).

Argument marshalling only: torch CUDA tensors are passed as raw device
pointers on the current HIP stream; every step of the search runs in the
library's kernels.  Importing this module fails loudly when the library has
not been built (``python -m paper_1304_4327_amd.build``); there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libknn_dualtree.so")

KNN_OK = 0
KNN_E_INVALID_ARG = 1
KNN_E_NONFINITE = 2
KNN_E_OOM = 3
KNN_E_DEVICE = 4
KNN_E_MODEL = 5
KNN_E_UNSUPPORTED = 6

KNN_BOUND_B = 0
KNN_BOUND_B1 = 1
KNN_BOUND_NONE = 2
KNN_PREC_FP32 = 0
KNN_PREC_BF16 = 1

BOUNDS = {"B": KNN_BOUND_B, "B1": KNN_BOUND_B1, "none": KNN_BOUND_NONE}
PRECISIONS = {"fp32": KNN_PREC_FP32, "bf16": KNN_PREC_BF16}


class KnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class knn_stats(ctypes.Structure):
    _fields_ = [("score_calls", ctypes.c_int64), ("leaf_tiles", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("inserts", ctypes.c_int64),
                ("fallback_leaves", ctypes.c_int64), ("fallback_queries", ctypes.c_int64),
                ("ms_query_build", ctypes.c_float), ("ms_search", ctypes.c_float),
                ("ms_main_kernel", ctypes.c_float), ("n_query_leaves", ctypes.c_int32),
                ("fallback_pairs", ctypes.c_int64), ("ms_ref_build", ctypes.c_float)]


class knn_opts(ctypes.Structure):
    _fields_ = [("bound", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("exclude_self", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed_radius", ctypes.c_void_p), ("leaf_kth_out", ctypes.c_void_p),
                ("stats", ctypes.POINTER(knn_stats))]


class knn_tree_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("dp", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("first_leaf", ctypes.c_int64), ("points", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("node_range", ctypes.c_void_p),
                ("box", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("split_dim", ctypes.c_void_p), ("ms_build", ctypes.c_float)]


# every symbol include/knn.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "knn_opts_default": (None, [ctypes.POINTER(knn_opts)]),
    "knn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "knn_last_error": (ctypes.c_char_p, []),
    "knn_release_cached_memory": (ctypes.c_int, []),
    "knn_cached_bytes": (ctypes.c_int64, []),
    "knn_build_tree": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P,
                                      ctypes.POINTER(_P)]),
    "knn_build_tree_pair": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "knn_free_tree": (None, [_P]),
    "knn_tree_get_info": (ctypes.c_int, [_P, ctypes.POINTER(knn_tree_info)]),
    "knn_search": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(knn_opts), _P, _P, _P]),
    "knn_search_points": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.POINTER(knn_opts), _P, _P, _P]),
    "knn_all_knn": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(knn_opts), _P,
                                   _P, _P]),
    "knn_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "knn_mlp_free": (None, [_P]),
    "knn_mlp_num_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "knn_mlp_set_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "knn_mlp_get_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "knn_mlp_get_grads": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "knn_mlp_set_norm": (ctypes.c_int, [_P, _P, _P, ctypes.c_float, ctypes.c_float]),
    "knn_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "knn_mlp_loss_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_float), _P]),
    "knn_mlp_adam_step": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, _P]),
    "knn_mlp_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "knn_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "knn_seed_features": (ctypes.c_int, [_P, _P, _P, _P]),
    "knn_seed_radius": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_float, _P, _P]),
    "knn_seed_train": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, _P,
                                      ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_float), _P, _P]),
    "knn_search_furthest": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(knn_opts), _P,
                                           _P, _P]),
    "knn_range_count": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(knn_opts), _P, ctypes.POINTER(ctypes.c_int64),
                                       _P]),
    "knn_range_fill": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(knn_opts), _P, _P, _P, _P]),
    "knn_kde": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(knn_opts),
                               _P, _P]),
    "knn_emst": (ctypes.c_int, [_P, ctypes.POINTER(knn_opts), _P, _P, _P,
                                ctypes.POINTER(ctypes.c_int32), _P]),
    "knn_search_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(knn_opts), _P,
                                          _P, _P]),
    "knn_debug_search_log": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(knn_opts),
                                            ctypes.c_int32, _P, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), _P, _P, _P]),
    "knn_debug_tile_replay": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(knn_opts),
                                             _P, _P, ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(ctypes.c_int64), _P]),
    "knn_debug_bf16_tiles": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P,
                                            _P, _P]),
}

_lib = None


def load():
    """Load the library (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_1304_4327_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != KNN_OK:
        msg = load().knn_last_error().decode()
        raise KnnError(status, msg)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2:
        raise TypeError(f"{name} must be a contiguous 2-D float32 tensor")
    return t


def _n_leaves_for(n: int, leaf_size: int) -> int:
    """Leaves of the tree the library builds over n points (complete tree of
    the smallest depth L with ceil(n / 2^L) <= leaf_size)."""
    L = 0
    while -(-n // (1 << L)) > leaf_size:
        L += 1
    return 1 << L


def _outputs(out, nq: int, k: int):
    """(idx, dist) output tensors: new ones, or the caller's after checking
    that the library may write n_q x k entries into them."""
    torch = _torch()
    if out is None:
        return (torch.empty((nq, k), dtype=torch.int64, device="cuda"),
                torch.empty((nq, k), dtype=torch.float32, device="cuda"))
    idx, dist = out
    for t, dt, nm in ((idx, torch.int64, "idx"), (dist, torch.float32, "dist")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"out {nm} must be a CUDA (HIP) tensor")
        if t.dtype != dt or not t.is_contiguous() or tuple(t.shape) != (nq, k):
            raise ValueError(f"out {nm} must be a contiguous {dt} tensor of shape ({nq}, {k}), "
                             f"got {t.dtype} {tuple(t.shape)}")
    return idx, dist


def _leaf_vec(t, n_leaves: int, name: str):
    """A per-query-leaf float32 vector the library reads or writes."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n_leaves:
        raise ValueError(f"{name} must be a contiguous float32 tensor with one entry per query "
                         f"leaf ({n_leaves}), got {t.dtype} with {t.numel()} entries")
    return t


class Tree:
    """Owning wrapper of a ``knn_tree*`` handle."""

    def __init__(self, handle, n, d):
        self.handle = handle
        self.n = n
        self.d = d

    def info(self):
        return knn_tree_get_info(self)

    def close(self):
        if self.handle:
            load().knn_free_tree(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def knn_build_tree(points, leaf_size: int, stream=None) -> Tree:
    """Build a kd-tree over ``points`` (CUDA float32 [n, d])."""
    if not hasattr(points, "is_cuda"):
        raise TypeError("points must be a CUDA tensor")
    _dev_f32(points, "points")
    out = ctypes.c_void_p()
    _check(load().knn_build_tree(ctypes.c_void_p(points.data_ptr()), points.shape[0],
                                 points.shape[1], int(leaf_size), _stream(stream),
                                 ctypes.byref(out)))
    return Tree(out, points.shape[0], points.shape[1])


def knn_release_cached_memory() -> None:
    """Return the library's cached device blocks to the runtime."""
    _check(load().knn_release_cached_memory())


def knn_cached_bytes() -> int:
    return int(load().knn_cached_bytes())


def knn_build_tree_pair(ref_points, query_points, leaf_size: int, stream=None):
    """Build the reference and the query kd-tree with overlapping builds;
    returns (reference Tree, query Tree)."""
    for x, nm in ((ref_points, "ref_points"), (query_points, "query_points")):
        if not hasattr(x, "is_cuda"):
            raise TypeError(f"{nm} must be a CUDA tensor")
        _dev_f32(x, nm)
    if ref_points.shape[1] != query_points.shape[1]:
        raise ValueError("ref_points and query_points differ in d")
    ra, qa = ctypes.c_void_p(), ctypes.c_void_p()
    _check(load().knn_build_tree_pair(ctypes.c_void_p(ref_points.data_ptr()), ref_points.shape[0],
                                      ctypes.c_void_p(query_points.data_ptr()),
                                      query_points.shape[0], ref_points.shape[1], int(leaf_size),
                                      _stream(stream), ctypes.byref(ra), ctypes.byref(qa)))
    return (Tree(ra, ref_points.shape[0], ref_points.shape[1]),
            Tree(qa, query_points.shape[0], query_points.shape[1]))


def knn_tree_get_info(tree: Tree) -> dict:
    info = knn_tree_info()
    _check(load().knn_tree_get_info(tree.handle, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in knn_tree_info._fields_}


def _make_opts(bound, precision, exclude_self, seed_radius, leaf_kth_out, stats):
    o = knn_opts()
    load().knn_opts_default(ctypes.byref(o))
    o.bound = BOUNDS[bound] if isinstance(bound, str) else int(bound)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.exclude_self = int(bool(exclude_self))
    o.seed_radius = seed_radius.data_ptr() if seed_radius is not None else None
    o.leaf_kth_out = leaf_kth_out.data_ptr() if leaf_kth_out is not None else None
    st = knn_stats() if stats else None
    o.stats = ctypes.pointer(st) if st is not None else None
    return o, st


def _stats_dict(st):
    if st is None:
        return None
    return {f: getattr(st, f) for f, _ in knn_stats._fields_}


def knn_search(ref: Tree, query: Tree | None, k: int, bound="B", precision="fp32",
               exclude_self=False, seed_radius=None, leaf_kth_out=None, stats=False,
               out=None, stream=None):
    """k nearest neighbours of every query point (query None: ref on itself).

    Returns (idx int64 [n_q, k], dist float32 [n_q, k], stats dict or None).
    ``seed_radius``/``leaf_kth_out`` are CUDA float32 tensors with one entry
    per query leaf.
    """
    qt = query or ref
    nq = qt.n
    idx, dist = _outputs(out, nq, k)
    if seed_radius is not None or leaf_kth_out is not None:
        nl = knn_tree_get_info(qt)["n_leaves"]
        _leaf_vec(seed_radius, nl, "seed_radius")
        _leaf_vec(leaf_kth_out, nl, "leaf_kth_out")
    o, st = _make_opts(bound, precision, exclude_self, seed_radius, leaf_kth_out, stats)
    _check(load().knn_search(ref.handle, query.handle if query is not None else None, int(k),
                             ctypes.byref(o), ctypes.c_void_p(idx.data_ptr()),
                             ctypes.c_void_p(dist.data_ptr()), _stream(stream)))
    return idx, dist, _stats_dict(st)


def knn_search_furthest(ref: Tree, query: Tree | None, k: int, bound="B", exclude_self=False,
                        stats=False, out=None, stream=None):
    """The k FARTHEST reference points of every query point (query None: ref
    on itself).  Returns (idx int64 [n_q, k], dist float32 [n_q, k]
    descending, stats dict or None)."""
    qt = query or ref
    idx, dist = _outputs(out, qt.n, k)
    o, st = _make_opts(bound, "fp32", exclude_self, None, None, stats)
    _check(load().knn_search_furthest(ref.handle, query.handle if query is not None else None,
                                      int(k), ctypes.byref(o), ctypes.c_void_p(idx.data_ptr()),
                                      ctypes.c_void_p(dist.data_ptr()), _stream(stream)))
    return idx, dist, _stats_dict(st)


def knn_range_search(ref: Tree, query: Tree | None, lo: float, hi: float, bound="B",
                     exclude_self=False, stats=False, stream=None):
    """Every reference point at a distance in [lo, hi] of each query point.
    Returns (offsets int64 [n_q + 1], idx int64 [total], dist float32
    [total], (count stats, fill stats) or None): the neighbours of query i
    are idx[offsets[i]:offsets[i+1]]."""
    torch = _torch()
    qt = query or ref
    qh = query.handle if query is not None else None
    offsets = torch.empty(qt.n + 1, dtype=torch.int64, device="cuda")
    total = ctypes.c_int64()
    o1, st1 = _make_opts(bound, "fp32", exclude_self, None, None, stats)
    _check(load().knn_range_count(ref.handle, qh, float(lo), float(hi), ctypes.byref(o1),
                                  ctypes.c_void_p(offsets.data_ptr()), ctypes.byref(total),
                                  _stream(stream)))
    idx = torch.empty(max(total.value, 1), dtype=torch.int64, device="cuda")
    dist = torch.empty(max(total.value, 1), dtype=torch.float32, device="cuda")
    o2, st2 = _make_opts(bound, "fp32", exclude_self, None, None, stats)
    _check(load().knn_range_fill(ref.handle, qh, float(lo), float(hi), ctypes.byref(o2),
                                 ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                                 _stream(stream)))
    st = (_stats_dict(st1), _stats_dict(st2)) if stats else None
    return offsets, idx[:total.value], dist[:total.value], st


def knn_kde(ref: Tree, query: Tree | None, h: float, eps: float, bound="B", exclude_self=False,
            stats=False, stream=None):
    """Gaussian kernel sums f(q) = sum_r exp(-|q - r|^2 / 2h^2) within eps per
    query.  Returns (f float64 [n_q], stats dict or None)."""
    torch = _torch()
    qt = query or ref
    f = torch.empty(qt.n, dtype=torch.float64, device="cuda")
    o, st = _make_opts(bound, "fp32", exclude_self, None, None, stats)
    _check(load().knn_kde(ref.handle, query.handle if query is not None else None, float(h),
                          float(eps), ctypes.byref(o), ctypes.c_void_p(f.data_ptr()),
                          _stream(stream)))
    return f, _stats_dict(st)


def knn_emst(tree: Tree, bound="B", stats=False, stream=None):
    """Euclidean minimum spanning tree of the tree's points (dual-tree
    Boruvka).  Returns (u int64 [n-1], v int64, w float32, rounds, stats
    dict or None) with u < v original rows."""
    torch = _torch()
    m = max(tree.n - 1, 1)
    u = torch.empty(m, dtype=torch.int64, device="cuda")
    v = torch.empty(m, dtype=torch.int64, device="cuda")
    w = torch.empty(m, dtype=torch.float32, device="cuda")
    rounds = ctypes.c_int32()
    o, st = _make_opts(bound, "fp32", False, None, None, stats)
    _check(load().knn_emst(tree.handle, ctypes.byref(o), ctypes.c_void_p(u.data_ptr()),
                           ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                           ctypes.byref(rounds), _stream(stream)))
    k = tree.n - 1
    return u[:k], v[:k], w[:k], rounds.value, _stats_dict(st)


def knn_search_noalloc(ref: Tree, query: Tree | None, k: int, out, bound="B", precision="fp32",
                       exclude_self=False, seed_radius=None, stats=False, stream=None):
    """knn_search without device allocation: the caller passes the outputs
    (idx int64 [n_q, k], dist float32 [n_q, k]); the library's scratch is a
    fixed per-device array (query trees of up to 2^18 leaves)."""
    if out is None:
        raise ValueError("knn_search_noalloc needs caller-allocated outputs (out=(idx, dist))")
    qt = query or ref
    idx, dist = _outputs(out, qt.n, k)
    if seed_radius is not None:
        _leaf_vec(seed_radius, knn_tree_get_info(qt)["n_leaves"], "seed_radius")
    o, st = _make_opts(bound, precision, exclude_self, seed_radius, None, stats)
    _check(load().knn_search_noalloc(ref.handle, query.handle if query is not None else None,
                                     int(k), ctypes.byref(o), ctypes.c_void_p(idx.data_ptr()),
                                     ctypes.c_void_p(dist.data_ptr()), _stream(stream)))
    return idx, dist, _stats_dict(st)


def knn_search_points(ref: Tree, queries, k: int, bound="B", precision="fp32",
                      seed_radius=None, leaf_kth_out=None, stats=False, out=None,
                      stream=None):
    """Build the query tree from ``queries`` (CUDA float32) and search."""
    _dev_f32(queries, "queries")
    nq = queries.shape[0]
    idx, dist = _outputs(out, nq, k)
    if seed_radius is not None or leaf_kth_out is not None:
        nl = _n_leaves_for(nq, knn_tree_get_info(ref)["leaf_size"])
        _leaf_vec(seed_radius, nl, "seed_radius")
        _leaf_vec(leaf_kth_out, nl, "leaf_kth_out")
    o, st = _make_opts(bound, precision, False, seed_radius, leaf_kth_out, stats)
    _check(load().knn_search_points(ref.handle, ctypes.c_void_p(queries.data_ptr()), nq,
                                    int(k), ctypes.byref(o), ctypes.c_void_p(idx.data_ptr()),
                                    ctypes.c_void_p(dist.data_ptr()), _stream(stream)))
    return idx, dist, _stats_dict(st)


def knn_all_knn(ref_points, query_points, k: int, leaf_size: int, bound="B", precision="fp32",
                exclude_self=False, stats=False, out=None, stream=None):
    """Build both trees (overlapped), search and free them in one call, with
    one stream synchronisation (query_points None: ref_points on itself).

    Returns (idx int64 [n_q, k], dist float32 [n_q, k], stats dict or None);
    with stats, ``ms_ref_build``/``ms_query_build`` give the build times.
    """
    _dev_f32(ref_points, "ref_points")
    if query_points is not None:
        _dev_f32(query_points, "query_points")
        if query_points.shape[1] != ref_points.shape[1]:
            raise ValueError("ref_points and query_points differ in d")
    nq = (query_points if query_points is not None else ref_points).shape[0]
    idx, dist = _outputs(out, nq, k)
    o, st = _make_opts(bound, precision, exclude_self, None, None, stats)
    _check(load().knn_all_knn(ctypes.c_void_p(ref_points.data_ptr()), ref_points.shape[0],
                              ctypes.c_void_p(query_points.data_ptr()) if query_points is not None
                              else None, nq if query_points is not None else 0,
                              ref_points.shape[1], int(leaf_size), int(k), ctypes.byref(o),
                              ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                              _stream(stream)))
    return idx, dist, _stats_dict(st)


# ---------------------------------------------------------------------------
# reading a tree's device arrays back (tests)
# ---------------------------------------------------------------------------
def _copy_dev(ptr, nbytes, dtype, shape):
    torch = _torch()
    t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(ptr), nbytes, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return t.cpu().numpy().view(dtype).reshape(shape)


def tree_arrays(tree: Tree) -> dict:
    """Host copies of the tree's arrays (numpy)."""
    i = knn_tree_get_info(tree)
    n, dp, nn = i["n"], i["dp"], i["n_nodes"]
    rng = _copy_dev(i["node_range"], nn * 8, np.int32, (nn, 2))
    box = _copy_dev(i["box"], nn * 2 * dp * 4, np.float32, (nn, 2, dp))
    return dict(
        info=i,
        points=_copy_dev(i["points"], (n + 64) * dp * 4, np.float32, (n + 64, dp)),
        perm=_copy_dev(i["perm"], n * 4, np.int32, (n,)),
        start=rng[:, 0], count=rng[:, 1],
        lo=box[:, 0, :i["d"]], hi=box[:, 1, :i["d"]], box_pad=box[:, :, i["d"]:],
        lam=_copy_dev(i["lambda_"], nn * 4, np.float32, (nn,)),
        split_dim=_copy_dev(i["split_dim"], nn * 4, np.int32, (nn,)),
    )


# ---------------------------------------------------------------------------
# seed network
# ---------------------------------------------------------------------------
class Mlp:
    """Owning wrapper of a ``knn_mlp*`` (n_in -> 64 -> 64 -> 1 network)."""

    def __init__(self, n_in: int | None = None, handle=None):
        if handle is None:
            h = ctypes.c_void_p()
            _check(load().knn_mlp_create(int(n_in), 64, ctypes.byref(h)))
            handle = h
        self.handle = handle
        n = ctypes.c_int64()
        _check(load().knn_mlp_num_params(self.handle, ctypes.byref(n)))
        self.n_params = n.value

    @classmethod
    def load_file(cls, path: str) -> "Mlp":
        h = ctypes.c_void_p()
        _check(load().knn_mlp_load(path.encode(), ctypes.byref(h)))
        return cls(handle=h)

    def save(self, path: str):
        _check(load().knn_mlp_save(self.handle, path.encode()))

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(load().knn_mlp_set_params(self.handle, p.ctypes.data, p.size))

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        _check(load().knn_mlp_get_params(self.handle, p.ctypes.data, p.size))
        return p

    def get_grads(self):
        g = np.empty(self.n_params, np.float32)
        _check(load().knn_mlp_get_grads(self.handle, g.ctypes.data, g.size))
        return g

    def set_norm(self, mu, inv_sd, y_mu=0.0, y_sd=1.0):
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        isd = np.ascontiguousarray(inv_sd, dtype=np.float32)
        _check(load().knn_mlp_set_norm(self.handle, mu.ctypes.data, isd.ctypes.data,
                                       float(y_mu), float(y_sd)))

    def forward(self, x, stream=None):
        torch = _torch()
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(load().knn_mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                      ctypes.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def loss_grad(self, x, t, stream=None) -> float:
        loss = ctypes.c_float()
        _check(load().knn_mlp_loss_grad(self.handle, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                        ctypes.byref(loss), _stream(stream)))
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(load().knn_mlp_adam_step(self.handle, float(lr), float(beta1), float(beta2),
                                        float(eps), _stream(stream)))

    def close(self):
        if self.handle:
            load().knn_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def knn_seed_features(ref: Tree, query: Tree | None, stream=None):
    """(n_query_leaves, d + 3) float32 CUDA tensor of seed features."""
    torch = _torch()
    qt = query or ref
    nl = knn_tree_get_info(qt)["n_leaves"]
    f = torch.empty((nl, ref.d + 3), dtype=torch.float32, device="cuda")
    _check(load().knn_seed_features(ref.handle, query.handle if query is not None else None,
                                    ctypes.c_void_p(f.data_ptr()), _stream(stream)))
    return f


def knn_seed_radius(mlp: Mlp, feats, log_margin: float = 0.0, stream=None):
    torch = _torch()
    r = torch.empty(feats.shape[0], dtype=torch.float32, device="cuda")
    _check(load().knn_seed_radius(mlp.handle, ctypes.c_void_p(feats.data_ptr()), feats.shape[0],
                                  float(log_margin), ctypes.c_void_p(r.data_ptr()),
                                  _stream(stream)))
    return r


class knn_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("val_frac", ctypes.c_float), ("target_fallback", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


def knn_seed_train(feats, kth, epochs: int = 30, batch: int = 4096, lr: float = 3e-3,
                   val_frac: float = 0.1, target_fallback: float = 0.05, seed: int = 0,
                   stream=None):
    """Train a seed network on the GPU (knn_seed_train in include/knn.h).
    feats: contiguous CUDA float32 (n, n_in); kth: contiguous CUDA float32
    (n,) per-leaf largest k-th distances.  Returns (Mlp, log_margin, list of
    per-epoch mean losses)."""
    torch = _torch()
    if feats.dim() != 2 or kth.dim() != 1 or kth.shape[0] != feats.shape[0]:
        raise ValueError("need feats (n, n_in) and kth (n,)")
    for t, nm in ((feats, "feats"), (kth, "kth")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous CUDA float32 tensor")
    o = knn_train_opts(int(epochs), int(batch), float(lr), float(val_frac),
                       float(target_fallback), int(seed) & 0xFFFFFFFFFFFFFFFF)
    h = ctypes.c_void_p()
    margin = ctypes.c_float()
    losses = np.zeros(int(epochs), np.float32) if epochs > 0 else np.zeros(1, np.float32)
    _check(load().knn_seed_train(ctypes.c_void_p(feats.data_ptr()), ctypes.c_void_p(kth.data_ptr()),
                                 feats.shape[0], feats.shape[1], ctypes.byref(o), ctypes.byref(h),
                                 ctypes.byref(margin), losses.ctypes.data, _stream(stream)))
    return Mlp(handle=h), margin.value, [float(v) for v in losses]


# ---------------------------------------------------------------------------
# test exports
# ---------------------------------------------------------------------------
def knn_debug_bf16_tiles(q, r, centre, stream=None):
    """BF16 tiles as the matrix-core kernels compute them.  q, r: CUDA
    float32 [n_tiles, 32, d]; centre: [n_tiles, d].  Returns (acc [n,32,32]
    indexed [tile, ref row, query], qnorm [n,32], margin [n,32])."""
    torch = _torch()
    n, rows, d = q.shape
    if rows != 32 or tuple(r.shape) != (n, 32, d) or tuple(centre.shape) != (n, d):
        raise ValueError("need q, r of shape (n, 32, d) and centre of shape (n, d)")
    for t, nm in ((q, "q"), (r, "r"), (centre, "centre")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous CUDA float32 tensor")
    acc = torch.empty((n, 32, 32), dtype=torch.float32, device="cuda")
    qn = torch.empty((n, 32), dtype=torch.float32, device="cuda")
    mg = torch.empty((n, 32), dtype=torch.float32, device="cuda")
    _check(load().knn_debug_bf16_tiles(ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(centre.data_ptr()), n, d,
                                       ctypes.c_void_p(acc.data_ptr()),
                                       ctypes.c_void_p(qn.data_ptr()),
                                       ctypes.c_void_p(mg.data_ptr()), _stream(stream)))
    return acc, qn, mg


DBG_WORDS = 12


def knn_debug_search_log(ref: Tree, query: Tree | None, k: int, bound="B", exclude_self=False,
                         far_first=False, capacity=1 << 20, stream=None):
    """knn_search through the debug kernel (d = 3): returns (idx, dist, log
    [n_records, 12] uint32 numpy, n_records).  The log holds one record per
    Score call (see knn_debug_search_log in include/knn.h)."""
    torch = _torch()
    nq = (query or ref).n
    idx, dist = _outputs(None, nq, k)
    log = torch.zeros((max(1, capacity), DBG_WORDS), dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    o, _ = _make_opts(bound, "fp32", exclude_self, None, None, False)
    _check(load().knn_debug_search_log(ref.handle, query.handle if query is not None else None,
                                       int(k), ctypes.byref(o), int(bool(far_first)),
                                       ctypes.c_void_p(log.data_ptr()), int(capacity),
                                       ctypes.byref(n), ctypes.c_void_p(idx.data_ptr()),
                                       ctypes.c_void_p(dist.data_ptr()), _stream(stream)))
    kept = min(n.value, capacity)
    return idx, dist, log[:kept].cpu().numpy().view(np.uint32), n.value


def knn_debug_tile_replay(ref: Tree, query: Tree | None, k: int, exclude_self=False, stream=None):
    """The search's BaseCase tiles replayed without the walk (d = 3 FP32).
    Returns (idx, dist, ms_search, ms_replay, pairs)."""
    nq = (query or ref).n
    idx, dist = _outputs(None, nq, k)
    ms_s, ms_r, pairs = ctypes.c_float(), ctypes.c_float(), ctypes.c_int64()
    o, _ = _make_opts("B", "fp32", exclude_self, None, None, False)
    _check(load().knn_debug_tile_replay(ref.handle, query.handle if query is not None else None,
                                        int(k), ctypes.byref(o), ctypes.c_void_p(idx.data_ptr()),
                                        ctypes.c_void_p(dist.data_ptr()), ctypes.byref(ms_s),
                                        ctypes.byref(ms_r), ctypes.byref(pairs), _stream(stream)))
    return idx, dist, ms_s.value, ms_r.value, pairs.value
