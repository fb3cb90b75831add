"""Training and use of the learned seed radius (host orchestration).

The network, its gradients and the Adam updates run in the library's kernels
(``knn_mlp_*``); the search consumes the predicted radii through
``knn_opts.seed_radius``.  This module only moves data: it runs plain
searches to collect per-query-leaf targets, standardises inputs and targets
(means and deviations computed on the host), feeds mini-batches, and
calibrates an additive log-margin on a held-out split.

Target of a query leaf: log of the largest k-th neighbour distance among its
points (the smallest seed for which the leaf needs no fallback).  Features:
leaf box centre, lambda, point count, log density of the reference leaf
reached from the centre (``knn_seed_features``).
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
    """Plain search on (ref, q) -> (features tensor, log-target tensor, stats)."""
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
    y = torch.from_numpy(np.log(np.maximum(kth.cpu().numpy().astype(np.float64), 1e-30))
                         .astype(np.float32)).cuda()
    return feats, y, st


def fit(feats_list, y_list, epochs: int = 30, batch: int = 4096, lr: float = 3e-3,
        seed: int = 0, val_frac: float = 0.1, target_fallback: float = 0.05) -> SeedModel:
    """Train the seed network on stacked (features, log-target) pairs."""
    import torch
    X = torch.cat(list(feats_list)).contiguous()
    Y = torch.cat(list(y_list)).contiguous()
    n = X.shape[0]
    order = np.random.default_rng(seed).permutation(n)
    n_val = max(1, int(n * val_frac))
    val_idx = torch.from_numpy(order[:n_val]).cuda()
    tr_idx = torch.from_numpy(order[n_val:]).cuda()
    Xtr, Ytr = X[tr_idx].contiguous(), Y[tr_idx]
    Xva, Yva = X[val_idx].contiguous(), Y[val_idx]
    xh = Xtr.double().cpu().numpy()
    yh = Ytr.double().cpu().numpy()
    mu = xh.mean(axis=0)
    sd = xh.std(axis=0)
    sd[sd < 1e-12] = 1.0
    y_mu, y_sd = float(yh.mean()), float(max(yh.std(), 1e-12))
    Ttr = torch.from_numpy(((yh - y_mu) / y_sd).astype(np.float32)).cuda()

    n_in = X.shape[1]
    mlp = K.Mlp(n_in)
    mlp.set_params(datagen.mlp_init(n_in, 64, seed))
    mlp.set_norm(mu.astype(np.float32), (1.0 / sd).astype(np.float32), y_mu, y_sd)
    history = []
    for ep in range(epochs):
        losses = []
        for bi in datagen.batches(Xtr.shape[0], batch, seed * 100003 + ep):
            idx = torch.from_numpy(bi).cuda()
            xb = Xtr[idx].contiguous()
            tb = Ttr[idx].contiguous()
            losses.append(mlp.loss_grad(xb, tb))
            mlp.adam_step(lr)
        history.append(float(np.mean(losses)))
    # calibration: residual quantile on the held-out split
    pred = mlp.forward(Xva).double().cpu().numpy() * y_sd + y_mu
    resid = Yva.double().cpu().numpy() - pred
    log_margin = float(np.quantile(resid, 1.0 - target_fallback))
    return SeedModel(mlp, log_margin, history)


def radii(model: SeedModel, feats):
    """Per-leaf seed radii (CUDA float32)."""
    return K.knn_seed_radius(model.mlp, feats, model.log_margin)


def train_for_workload(name: str, train_seeds, scale: float = 1.0, precision: str = "fp32",
                       **kw) -> SeedModel:
    """Targets come from plain (exact) searches on the training seeds; the
    precision only picks which exact path produces them."""
    feats, ys = [], []
    for s in train_seeds:
        ref, q, k, leaf = datagen.make(name, seed=s, scale=scale)
        f, y, _ = leaf_data(ref, q, k, leaf, precision=precision)
        feats.append(f)
        ys.append(y)
    return fit(feats, ys, **kw)
