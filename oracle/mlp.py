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


# ---- training procedure --------------------------------------------------
# The steps of the library's seed training, in FP64, with the random numbers
# drawn from SplitMix64 (Steele, Lea and Flood, 2014) in counter form:
# value(s, i) = mix(s + (i + 1) * 0x9E3779B97F4A7C15) mod 2^64; stream p
# (0 weights, 1 split, 2 + e epoch e) is seeded with value(seed, p).

_GOLDEN = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def splitmix_values(s: int, count: int) -> np.ndarray:
    """Values 0 .. count-1 of the SplitMix64 sequence that starts at state s
    (Python integers, exact modulo 2^64)."""
    out = np.empty(count, np.uint64)
    for i in range(count):
        z = (s + (i + 1) * _GOLDEN) & _MASK
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out[i] = z ^ (z >> 31)
    return out


def splitmix_value(s: int, i: int) -> int:
    return int(splitmix_values((s + i * _GOLDEN) & _MASK, 1)[0])


def key_order(s: int, n: int) -> np.ndarray:
    """Rows 0 .. n-1 ordered by (key, row), key i = value i of stream s."""
    keys = splitmix_values(s, n)
    return np.lexsort((np.arange(n), keys))


def init_params(n_in: int, H: int, seed: int) -> np.ndarray:
    """Weights uniform in +-sqrt(6 / fan_in) from stream 0 (one counter over
    W1, W2, w3 in that order), biases zero; FP32 values as the library
    stores them."""
    s0 = splitmix_value(seed, 0)
    n_w = H * n_in + H * H + H
    u = (splitmix_values(s0, n_w) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    parts, at = [], 0
    for fan_out, fan_in in ((H, n_in), (H, H), (1, H)):
        a = np.sqrt(6.0 / fan_in)
        parts.append((-a + 2.0 * a * u[at:at + fan_out * fan_in]).astype(np.float32))
        parts.append(np.zeros(fan_out, np.float32))
        at += fan_out * fan_in
    return np.concatenate(parts).astype(np.float64)


def train(feats, kth, epochs, batch, lr, val_frac, target_fallback, seed, H=64):
    """The seed training in FP64.  Returns (params, mu, inv_sd, y_mu, y_sd,
    log_margin, per-epoch mean losses).

    1. rows ordered by random key (stream 1): the first max(1, floor(n *
       val_frac)) are held out;
    2. mean and population deviation of every training column (deviation
       below 1e-12 counts as 1), targets t = (log max(kth, 1e-30) - y_mu) /
       y_sd;
    3. initial weights from stream 0;
    4. each epoch e: training rows in the key order of stream 2 + e, cut into
       batches; mean squared error gradient and one Adam step per batch;
    5. log margin: the (1 - target_fallback) quantile, linear between order
       statistics, of the held-out residuals log kth - (y * y_sd + y_mu).
    """
    x = np.asarray(feats, np.float64)
    y = np.log(np.maximum(np.asarray(kth, np.float64), 1e-30))
    n, n_in = x.shape
    n_val = max(1, int(np.floor(n * val_frac)))
    order = key_order(splitmix_value(seed, 1), n)
    va, tr = order[:n_val], order[n_val:]
    xtr, ytr = x[tr], y[tr]
    mu = xtr.mean(axis=0)
    sd = xtr.std(axis=0)
    sd[sd < 1e-12] = 1.0
    y_mu, y_sd = float(ytr.mean()), max(float(ytr.std()), 1e-12)
    t = (ytr - y_mu) / y_sd
    inv_sd = 1.0 / sd
    p = init_params(n_in, H, seed)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    step = 0
    history = []
    for e in range(epochs):
        o = key_order(splitmix_value(seed, 2 + e), len(tr))
        losses = []
        for b0 in range(0, len(tr), batch):
            bi = o[b0:b0 + batch]
            L, g = loss_and_grad(p, xtr[bi], t[bi], mu, inv_sd, n_in, H)
            step += 1
            p, m, v = adam_step(p, g, m, v, step, lr)
            losses.append(L)
        history.append(float(np.mean(losses)))
    pred = forward(p, x[va], mu, inv_sd, n_in, H) * y_sd + y_mu
    resid = y[va] - pred
    margin = float(np.quantile(resid, 1.0 - target_fallback))
    return p, mu, inv_sd, y_mu, y_sd, margin, history
