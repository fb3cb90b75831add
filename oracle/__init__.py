"""CPU oracle for the exact k-NN dual-tree search -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything here.  The GPU library never calls into this
package and shares no code, header, table or helper with it; the two meet
only through the seeded input generators (``paper_1304_4327_amd.datagen``),
which draw random numbers and hold none of the method's arithmetic.

Modules
-------
knn      FP64 brute-force k-NN (C, OpenMP) -- the definition the dual-tree
         method reaches exactly (k-NN problem statement and brute-force
         remark, Section "k-Nearest Neighbor Search").
kdtree   plain recursive kd-tree build with the split rule the GPU build
         follows, plus the node quantities (box, centre, lambda) of
         Section "Space Trees".
dualtree slow, literal pruning dual-tree traversal (Algorithms 1-3) for tiny
         inputs, used to pin the reading of the bound B(N_q).
mlp      FP64 forward / backward / Adam for the seed-radius network.
parity   the acceptance predicate comparing a GPU answer with the oracle.
"""
