"""FP64 reference for the seed-radius network (test infrastructure only).

The learned seed is not part of the paper: it only supplies an initial value
for the pruning bound of a query node, and any value keeps the search exact
(a query whose k-th distance exceeds its seed is searched again without it).
This module fixes what the GPU kernels compute, in the plainest form:

network   x_hat = (x - mu) * inv_sd           (fixed input standardisation)
          a1 = W1 x_hat + b1,  h1 = relu(a1)  (H units)
          a2 = W2 h1   + b2,   h2 = relu(a2)  (H units)
          y  = w3 . h2 + b3                   (one output)
loss      L = (1/n) sum_i (y_i - t_i)^2
gradient  by the chain rule; relu'(a) = 1 if a > 0 else 0
optimiser Adam with bias correction (Kingma and Ba):
          m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
          p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Parameters travel as one flat vector in the order W1 (H x n_in, row-major),
b1 (H), W2 (H x H, row-major), b2 (H), w3 (H), b3 (1).
"""
from __future__ import annotations

import numpy as np


def n_params(n_in: int, H: int) -> int:
    return H * n_in + H + H * H + H + H + 1


def unpack(p, n_in: int, H: int):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3.ravel(), np.ravel(b3)])


def forward(p, x, mu, inv_sd, n_in, H, keep=False):
    W1, b1, W2, b2, w3, b3 = unpack(p, n_in, H)
    xh = (np.asarray(x, np.float64) - mu) * inv_sd
    a1 = xh @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3 + b3[0]
    if keep:
        return y, (xh, a1, h1, a2, h2)
    return y


def loss_and_grad(p, x, t, mu, inv_sd, n_in, H):
    W1, b1, W2, b2, w3, b3 = unpack(p, n_in, H)
    y, (xh, a1, h1, a2, h2) = forward(p, x, mu, inv_sd, n_in, H, keep=True)
    t = np.asarray(t, np.float64)
    n = y.shape[0]
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    g_w3 = h2.T @ dy
    g_b3 = np.array([dy.sum()])
    da2 = np.outer(dy, w3) * (a2 > 0)
    g_W2 = da2.T @ h1
    g_b2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    g_W1 = da1.T @ xh
    g_b1 = da1.sum(axis=0)
    return L, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (t >= 1).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
