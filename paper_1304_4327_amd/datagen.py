"""Seeded synthetic point sets for the k-NN workloads.

This module only draws random numbers: it holds none of the search's
arithmetic, so both the GPU path and the CPU oracle may take their inputs
from it.  Every generator works in FP64 with ``numpy.random.default_rng`` and
casts to FP32 once; queries and references are independent draws from the
same distribution parameters (independent child streams of one
``SeedSequence``: parameters, references, queries).

Workload recipes (sizes are arguments so tests can shrink them):

* ``uniform``   -- i.i.d. uniform on [0, 1)^d.
* ``gmm``       -- isotropic Gaussian mixture: means uniform in [0, 100)^d,
  per-component sigma log-uniform in [0.5, 5]; component weights equal, or
  Zipf-like (w_c proportional to c^-s) when ``zipf_s`` is given.
* ``manifold_tanh`` -- latent z uniform in [0, 1)^m, mapped by a shared
  random Gaussian m x d matrix and a tanh, plus N(0, noise^2) per coordinate.
* ``manifold_linear`` -- as above without the tanh (linear embedding).
* ``lattice``   -- integer grid points (closed-form neighbour sets).
"""
from __future__ import annotations

import numpy as np


def _streams(seed: int, n: int = 3):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, d)).astype(np.float32)


def _gmm_params(rng, d, n_comp, zipf_s):
    means = rng.uniform(0.0, 100.0, size=(n_comp, d))
    sig = np.exp(rng.uniform(np.log(0.5), np.log(5.0), size=n_comp))
    if zipf_s is None:
        w = np.full(n_comp, 1.0 / n_comp)
    else:
        w = np.arange(1, n_comp + 1, dtype=np.float64) ** (-float(zipf_s))
        w /= w.sum()
    return means, sig, w


def _gmm_draw(rng, n, means, sig, w):
    comp = rng.choice(len(w), size=n, p=w)
    x = means[comp] + sig[comp, None] * rng.standard_normal((n, means.shape[1]))
    return x.astype(np.float32)


def gmm_pair(n_ref: int, n_query: int, d: int, n_comp: int, seed: int,
             zipf_s: float | None = None):
    """Reference and query sets drawn from one Gaussian mixture."""
    pr, rr, qr = _streams(seed)
    means, sig, w = _gmm_params(pr, d, n_comp, zipf_s)
    return _gmm_draw(rr, n_ref, means, sig, w), _gmm_draw(qr, n_query, means, sig, w)


def _manifold(rng, n, A, noise, tanh):
    z = rng.random((n, A.shape[0]))
    x = z @ A
    if tanh:
        x = np.tanh(x)
    x = x + noise * rng.standard_normal(x.shape)
    return x.astype(np.float32)


def manifold_pair(n_ref: int, n_query: int, latent: int, d: int, noise: float,
                  seed: int, tanh: bool):
    pr, rr, qr = _streams(seed)
    A = pr.standard_normal((latent, d))
    return (_manifold(rr, n_ref, A, noise, tanh),
            _manifold(qr, n_query, A, noise, tanh))


def lattice(side: int, d: int) -> np.ndarray:
    axes = [np.arange(side, dtype=np.float32)] * d
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.ravel() for a in g], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# The five workloads.  ``scale`` shrinks the point counts (tests); 1.0 is the
# full size.  Each returns (reference, query_or_None, k, leaf_size); a None
# query set means all-kNN of the reference set on itself with the self match
# excluded.
# --------------------------------------------------------------------------
WORKLOADS = {
    "uniform10k_d3_k5": dict(n_ref=10_000, n_query=None, d=3, k=5, leaf=20),
    "gmm1m_d3_k10": dict(n_ref=1_000_000, n_query=1_000_000, d=3, k=10, leaf=32),
    "manifold4m_d16_k10": dict(n_ref=4_000_000, n_query=1_000_000, d=16, k=10, leaf=32),
    "zipfgmm2m_d8_k10": dict(n_ref=2_000_000, n_query=2_000_000, d=8, k=10, leaf=32),
    "manifold1m_d64_k50": dict(n_ref=1_000_000, n_query=262_144, d=64, k=50, leaf=32),
}

DEFAULT_SEEDS = {
    "uniform10k_d3_k5": 1,
    "gmm1m_d3_k10": 2,
    "manifold4m_d16_k10": 3,
    "zipfgmm2m_d8_k10": 48,       # held-out seed; training seeds are 40..47
    "manifold1m_d64_k50": 5,
}


def make(name: str, seed: int | None = None, scale: float = 1.0):
    cfg = WORKLOADS[name]
    seed = DEFAULT_SEEDS[name] if seed is None else seed
    nr = max(2, int(round(cfg["n_ref"] * scale)))
    nq = None if cfg["n_query"] is None else max(1, int(round(cfg["n_query"] * scale)))
    d = cfg["d"]
    if name.startswith("uniform"):
        ref, q = uniform(nr, d, seed), None
    elif name.startswith("gmm"):
        ref, q = gmm_pair(nr, nq, d, 32, seed)
    elif name.startswith("zipfgmm"):
        ref, q = gmm_pair(nr, nq, d, 64, seed, zipf_s=1.2)
    elif name.startswith("manifold4m"):
        ref, q = manifold_pair(nr, nq, 4, d, 0.01, seed, tanh=True)
    elif name.startswith("manifold1m"):
        ref, q = manifold_pair(nr, nq, 10, d, 0.02, seed, tanh=False)
    else:  # pragma: no cover
        raise KeyError(name)
    return ref, q, cfg["k"], cfg["leaf"]


def mlp_init(n_in: int, hidden: int, seed: int) -> np.ndarray:
    """Initial parameters of the seed network as one flat FP32 vector in the
    order W1 (hidden x n_in), b1, W2 (hidden x hidden), b2, w3 (hidden), b3:
    weights uniform in +-sqrt(6 / fan_in) (He), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((hidden, n_in), (hidden, hidden), (1, hidden)):
        a = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def batches(n: int, batch: int, epoch_seed: int):
    """A seeded random permutation of range(n) cut into mini-batches."""
    order = np.random.default_rng(epoch_seed).permutation(n)
    return [order[i:i + batch] for i in range(0, n, batch)]
