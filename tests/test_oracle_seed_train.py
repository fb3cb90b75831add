"""Pins for the FP64 seed-training procedure (oracle.mlp.train): the random
generator against SplitMix64's published test vector, the split and batch
orders as permutations, the initial weights' range, the standardisation
invariants, the calibrated margin's quantile property, and convergence on a
target the network can represent."""
import numpy as np
import pytest

from oracle import mlp


def test_splitmix_published_vector():
    # the first five outputs of SplitMix64 from state 1234567, as published
    # with the generator's reference implementation
    got = mlp.splitmix_values(1234567, 5)
    assert got.tolist() == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                            4593380528125082431, 16408922859458223821]
    # counter form: value(s, i) starts the sequence i steps later
    assert mlp.splitmix_value(1234567, 3) == 4593380528125082431


def test_key_order_is_a_permutation_sorted_by_key():
    o = mlp.key_order(99, 1000)
    assert sorted(o.tolist()) == list(range(1000))
    keys = mlp.splitmix_values(99, 1000)
    assert np.all(np.diff(keys[o].astype(np.float64)) >= 0)
    # another stream gives another order
    assert not np.array_equal(o, mlp.key_order(100, 1000))


@pytest.mark.parametrize("n_in", [1, 6, 11, 67])
def test_init_ranges_and_zero_biases(n_in):
    H = 64
    p = mlp.init_params(n_in, H, 5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, n_in, H)
    for w, fan_in in ((W1, n_in), (W2, H), (w3, H)):
        a = np.sqrt(6.0 / fan_in)
        assert np.all(np.abs(w) <= a)
        # uniform on [-a, a]: mean near 0, variance near a^2 / 3
        assert abs(w.mean()) < 4 * a / np.sqrt(3 * w.size)
        tol = 0.5 if w.size < 200 else 0.15
        assert abs(w.var() / (a * a / 3) - 1) < tol
    assert not b1.any() and not b2.any() and not b3.any()
    assert np.array_equal(p, p.astype(np.float32).astype(np.float64))


def _data(n=400, n_in=5, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n_in)) * rng.uniform(0.1, 10, n_in) + rng.normal(size=n_in) * 5
    # a target the network can represent: log kth linear in the features
    w = rng.normal(size=n_in) / (1 + np.abs(x).mean(axis=0))
    kth = np.exp(x @ w + 0.05 * rng.normal(size=n))
    return x, kth


def test_standardisation_and_split():
    x, kth = _data()
    p, mu, inv_sd, y_mu, y_sd, margin, hist = mlp.train(x, kth, 1, 64, 1e-3, 0.25, 0.1, 3)
    n_val = 100
    tr = mlp.key_order(mlp.splitmix_value(3, 1), 400)[n_val:]
    xs = (x[tr] - mu) * inv_sd
    assert np.allclose(xs.mean(axis=0), 0, atol=1e-12)
    assert np.allclose(xs.std(axis=0), 1, atol=1e-12)
    t = (np.log(kth[tr]) - y_mu) / y_sd
    assert abs(t.mean()) < 1e-12 and abs(t.std() - 1) < 1e-12
    # a constant column keeps unit scale
    xc = x.copy()
    xc[:, 2] = 7.0
    _, mu_c, isd_c, *_ = mlp.train(xc, kth, 1, 64, 1e-3, 0.25, 0.1, 3)
    assert mu_c[2] == 7.0 and isd_c[2] == 1.0


@pytest.mark.parametrize("target", [0.0, 0.1, 0.3])
def test_margin_is_the_held_out_quantile(target):
    x, kth = _data(seed=1)
    n_val = 120
    p, mu, inv_sd, y_mu, y_sd, margin, _ = mlp.train(x, kth, 2, 50, 3e-3, 0.3, target, 11)
    va = mlp.key_order(mlp.splitmix_value(11, 1), 400)[:n_val]
    resid = np.log(kth[va]) - (mlp.forward(p, x[va], mu, inv_sd, x.shape[1], 64) * y_sd + y_mu)
    above = np.mean(resid > margin + 1e-12)
    assert above <= target + 1e-12
    assert above >= target - 1.0 / (n_val - 1) - 1e-12
    if target == 0.0:
        assert margin == pytest.approx(resid.max(), abs=1e-12)


def test_training_fits_a_representable_target():
    x, kth = _data(n=600, seed=2)
    *_, hist = mlp.train(x, kth, 40, 64, 3e-3, 0.1, 0.05, 5)
    assert hist[-1] < 0.1 * hist[0]
    assert hist[-1] < 0.05
