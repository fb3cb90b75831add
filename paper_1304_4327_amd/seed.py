"""Training and use of the learned seed radius (host orchestration).

Training runs in the library (``knn_seed_train``: split, standardisation,
mini-batch gradients and Adam steps, margin calibration); the search consumes
the predicted radii through ``knn_opts.seed_radius``.  This module only runs
the plain searches that produce the training rows and stacks them.

Target of a query leaf: the largest k-th neighbour distance among its points
(the smallest seed for which the leaf needs no fallback); the network learns
its log.  Features: leaf box centre, lambda, point count, log density of the
reference leaf reached from the centre (``knn_seed_features``).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import datagen
from . import knn as K


@dataclasses.dataclass
class SeedModel:
    mlp: K.Mlp
    log_margin: float
    history: list


def leaf_data(ref_pts, q_pts, k: int, leaf: int, precision: str = "fp32"):
    """Plain search on (ref, q) -> (features, per-leaf k-th distances, stats),
    both CUDA float32 tensors."""
    import torch
    R = torch.from_numpy(np.ascontiguousarray(ref_pts)).cuda()
    rt = K.knn_build_tree(R, leaf)
    if q_pts is None:
        qt = None
        nl = rt.info()["n_leaves"]
    else:
        Q = torch.from_numpy(np.ascontiguousarray(q_pts)).cuda()
        qt = K.knn_build_tree(Q, leaf)
        nl = qt.info()["n_leaves"]
    kth = torch.empty(nl, dtype=torch.float32, device="cuda")
    _, _, st = K.knn_search(rt, qt, k, precision=precision, exclude_self=q_pts is None,
                            leaf_kth_out=kth, stats=True)
    feats = K.knn_seed_features(rt, qt)
    if qt is not None:
        qt.close()
    rt.close()
    return feats, kth, st


def fit(feats_list, kth_list, epochs: int = 30, batch: int = 4096, lr: float = 3e-3,
        seed: int = 0, val_frac: float = 0.1, target_fallback: float = 0.05) -> SeedModel:
    """Train the seed network on stacked (features, k-th distance) rows."""
    import torch
    X = torch.cat(list(feats_list)).contiguous()
    Y = torch.cat(list(kth_list)).contiguous()
    mlp, margin, history = K.knn_seed_train(X, Y, epochs=epochs, batch=batch, lr=lr,
                                            val_frac=val_frac, target_fallback=target_fallback,
                                            seed=seed)
    return SeedModel(mlp, margin, history)


def radii(model: SeedModel, feats):
    """Per-leaf seed radii (CUDA float32)."""
    return K.knn_seed_radius(model.mlp, feats, model.log_margin)


def train_for_workload(name: str, train_seeds, scale: float = 1.0, precision: str = "fp32",
                       **kw) -> SeedModel:
    """Targets come from plain (exact) searches on the training seeds; the
    precision only picks which exact path produces them."""
    feats, kths = [], []
    for s in train_seeds:
        ref, q, k, leaf = datagen.make(name, seed=s, scale=scale)
        f, kth, _ = leaf_data(ref, q, k, leaf, precision=precision)
        feats.append(f)
        kths.append(kth)
    return fit(feats, kths, **kw)
