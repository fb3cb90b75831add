"""Exact k-nearest-neighbour search by a pruning dual-tree traversal over
kd-trees, on AMD MI355X (gfx950).

The compute lives in a HIP shared library (``libknn_dualtree.so``, C ABI
declared in ``include/knn.h``); :mod:`paper_1304_4327_amd.knn` is the thin
ctypes binding with the same names.  Import submodules explicitly
(``from paper_1304_4327_amd import knn``) so that
:mod:`paper_1304_4327_amd.datagen` (seeded inputs only) stays importable
without the library.
"""
