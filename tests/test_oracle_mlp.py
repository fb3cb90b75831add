"""Pins for the FP64 seed-network reference: gradients by central finite
differences, Adam's first step in closed form, and special cases."""
import numpy as np

from oracle import mlp
from paper_1304_4327_amd import datagen


def _setup(n_in=5, H=8, n=13, seed=0):
    rng = np.random.default_rng(seed)
    p = datagen.mlp_init(n_in, H, seed).astype(np.float64)
    p[H * n_in:H * n_in + H] = rng.normal(0, 0.1, H)          # non-zero biases
    x = rng.normal(size=(n, n_in))
    t = rng.normal(size=n)
    mu = rng.normal(size=n_in)
    inv_sd = rng.uniform(0.5, 2.0, n_in)
    return p, x, t, mu, inv_sd, n_in, H


def test_gradient_matches_finite_differences():
    p, x, t, mu, isd, n_in, H = _setup()
    L, g = mlp.loss_and_grad(p, x, t, mu, isd, n_in, H)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, x, t, mu, isd, n_in, H)
        lm, _ = mlp.loss_and_grad(p - e, x, t, mu, isd, n_in, H)
        num[i] = (lp - lm) / (2 * h)
    scale = np.abs(g).max()
    assert np.all(np.abs(num - g) <= 1e-6 * (np.abs(g) + 1e-3 * scale))


def test_loss_is_mean_squared_error():
    p, x, t, mu, isd, n_in, H = _setup()
    y = mlp.forward(p, x, mu, isd, n_in, H)
    L, _ = mlp.loss_and_grad(p, x, t, mu, isd, n_in, H)
    assert np.isclose(L, np.mean((y - t) ** 2), rtol=1e-15)


def test_zero_hidden_weights_give_bias():
    n_in, H = 3, 4
    p = np.zeros(mlp.n_params(n_in, H))
    p[-1] = 2.5
    y = mlp.forward(p, np.ones((6, n_in)), np.zeros(n_in), np.ones(n_in), n_in, H)
    assert np.all(y == 2.5)


def test_single_unit_closed_form():
    """One active path: y = w3 * relu(w2 * relu(w1 * x + b1) + b2) + b3."""
    n_in, H = 1, 1
    p = mlp.pack(np.array([[2.0]]), np.array([-1.0]), np.array([[3.0]]), np.array([0.5]),
                 np.array([-1.5]), np.array([0.25]))
    x = np.array([[0.0], [1.0], [2.0]])
    y = mlp.forward(p, x, np.zeros(1), np.ones(1), n_in, H)
    want = [-1.5 * max(3 * max(2 * v - 1, 0) + 0.5, 0) + 0.25 for v in (0, 1, 2)]
    assert np.allclose(y, want, rtol=0, atol=0)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by -lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    lr, eps = 0.01, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr, 0.9, 0.999, eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(1)
    n_in, H = 4, 16
    x = rng.normal(size=(256, n_in))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2
    p = datagen.mlp_init(n_in, H, 3).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    mu, isd = np.zeros(n_in), np.ones(n_in)
    L0, _ = mlp.loss_and_grad(p, x, t, mu, isd, n_in, H)
    for step in range(1, 301):
        L, g = mlp.loss_and_grad(p, x, t, mu, isd, n_in, H)
        p, m, v = mlp.adam_step(p, g, m, v, step, 1e-2)
    assert L < 0.2 * L0
