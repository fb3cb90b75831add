"""The C-ABI library loads, exports every symbol include/knn.h declares,
and rejects bad arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1304_4327_amd import knn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "knn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knn_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = knn.load()
    names = _declared()
    assert "knn_search" in names and "knn_build_tree" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(knn._SIGS), "binding lacks a declared symbol"


def test_status_strings():
    lib = knn.load()
    assert lib.knn_status_string(0) == b"ok"
    assert lib.knn_status_string(knn.KNN_E_INVALID_ARG) == b"invalid argument"


def test_opts_default():
    o = knn.knn_opts()
    o.bound = 7
    knn.load().knn_opts_default(ctypes.byref(o))
    assert o.bound == knn.KNN_BOUND_B and o.precision == knn.KNN_PREC_FP32
    assert not o.seed_radius and o.exclude_self == 0


@pytest.mark.parametrize("n,d,leaf", [(0, 3, 8), (10, 0, 8), (10, 65, 8), (10, 3, 0),
                                      (10, 3, 65), (-5, 3, 8)])
def test_build_tree_rejects_bad_domain(n, d, leaf):
    lib = knn.load()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation comes first
    st = lib.knn_build_tree(fake, n, d, leaf, None, ctypes.byref(out))
    assert st == knn.KNN_E_INVALID_ARG
    assert lib.knn_last_error()
    assert not out.value


def test_build_tree_rejects_null_points():
    lib = knn.load()
    out = ctypes.c_void_p()
    assert lib.knn_build_tree(None, 10, 3, 8, None, ctypes.byref(out)) == knn.KNN_E_INVALID_ARG


@pytest.mark.parametrize("which", ["ref_null", "query_null", "query_n", "out_null"])
def test_build_tree_pair_rejects_bad_arguments(which):
    lib = knn.load()
    ra, qa = ctypes.c_void_p(), ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation comes first
    ref = None if which == "ref_null" else fake
    qry = None if which == "query_null" else fake
    nq = 0 if which == "query_n" else 10
    qout = None if which == "out_null" else ctypes.byref(qa)
    st = lib.knn_build_tree_pair(ref, 10, qry, nq, 3, 8, None, ctypes.byref(ra), qout)
    assert st == knn.KNN_E_INVALID_ARG
    assert lib.knn_last_error()
    assert not ra.value and not qa.value


@pytest.mark.parametrize("which", ["ref_null", "ref_n", "query_n", "bad_d", "bad_leaf"])
def test_all_knn_rejects_bad_arguments(which):
    # argument checks run before any device work (no GPU needed)
    lib = knn.load()
    o = knn.knn_opts()
    lib.knn_opts_default(ctypes.byref(o))
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation comes first
    ref = None if which == "ref_null" else fake
    nr = 0 if which == "ref_n" else 10
    nq = 0 if which == "query_n" else 10
    d = 0 if which == "bad_d" else 3
    leaf = 0 if which == "bad_leaf" else 8
    st = lib.knn_all_knn(ref, nr, fake, nq, d, leaf, 3, ctypes.byref(o), ctypes.c_void_p(8),
                         ctypes.c_void_p(8), None)
    assert st == knn.KNN_E_INVALID_ARG
    assert lib.knn_last_error()


def test_search_rejects_null_tree():
    lib = knn.load()
    o = knn.knn_opts()
    lib.knn_opts_default(ctypes.byref(o))
    st = lib.knn_search(None, None, 3, ctypes.byref(o), ctypes.c_void_p(8), ctypes.c_void_p(8),
                        None)
    assert st == knn.KNN_E_INVALID_ARG
    assert b"NULL" in lib.knn_last_error()


def test_binding_rejects_bad_output_and_leaf_tensors():
    """The binding checks every buffer the library writes or reads by raw
    pointer before the call (the C ABI cannot check device-buffer sizes)."""
    import torch
    cpu = torch.empty((4, 3), dtype=torch.int64)
    with pytest.raises(ValueError):
        knn._outputs((cpu, torch.empty((4, 3))), 4, 3)
    with pytest.raises(ValueError):
        knn._leaf_vec(torch.empty(8), 8, "seed_radius")
    assert knn._leaf_vec(None, 8, "seed_radius") is None


def test_leaf_count_rule():
    from oracle import kdtree as kd
    for n, leaf in [(1, 1), (5, 2), (10_000, 20), (1_000_000, 32), (262_144, 32), (33, 32)]:
        assert knn._n_leaves_for(n, leaf) == 1 << kd.depth_for(n, leaf)
