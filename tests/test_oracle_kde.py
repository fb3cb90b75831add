"""Pins of the kernel-density oracle (Section "Kernel Density Estimation",
Algorithms 9 and 10; Gaussian kernel K(d) = exp(-d^2 / 2h^2)): closed forms
(a lattice sum equals a Gaussian integral to far below FP64 precision, by
Poisson summation; a single reference point), the numpy form, the self
term, and the literal dual-tree estimate within its error bound eps (the
printed comparison is shown to break it)."""
import math

import numpy as np
import pytest

from oracle import dualtree as dt
from oracle import knn as ok
from paper_1304_4327_amd import datagen


def test_lattice_sum_closed_form():
    """sum over integers n of exp(-n^2 / (2 h^2)) = h sqrt(2 pi) (1 + 2 sum_k
    exp(-2 pi^2 h^2 k^2)); at h = 2 the correction is below 1e-33, so the
    1-D sum is sqrt(8 pi) and the 3-D lattice sum its cube (terms past |n|
    = 60 resp. 30 are below 1e-100)."""
    line = np.arange(-60, 61, dtype=np.float32)[:, None]
    f, _ = ok.kde(np.zeros((1, 1), np.float32), line, 2.0)
    assert abs(f[0] - math.sqrt(8 * math.pi)) < 1e-14 * f[0]
    cube = datagen.lattice(61, 3) - 30.0
    f, _ = ok.kde(np.zeros((1, 3), np.float32), cube, 2.0)
    assert abs(f[0] - math.sqrt(8 * math.pi) ** 3) < 1e-13 * f[0]
    # off-lattice query: shifted by half a step the sum is still the
    # integral (the correction alternates in sign but stays below 1e-33)
    f, _ = ok.kde(np.full((1, 1), 0.5, np.float32), line, 2.0)
    assert abs(f[0] - math.sqrt(8 * math.pi)) < 1e-14 * f[0]


def test_single_reference_and_self_term():
    r = np.array([[1.0, 2.0, 2.0]], np.float32)
    f, b = ok.kde(np.zeros((1, 3), np.float32), r, 1.5)
    assert f[0] == pytest.approx(math.exp(-9.0 / 4.5), rel=1e-15)
    assert b[0] == pytest.approx(math.exp(-2.0) * 3.0, rel=1e-15)
    x = datagen.uniform(300, 2, 3)
    full, _ = ok.kde(x, x, 0.2)
    loo, _ = ok.kde(x, x, 0.2, exclude_self=True)
    np.testing.assert_allclose(full - loo, 1.0, rtol=0, atol=1e-12)


def test_numpy_form_agrees():
    rng = np.random.default_rng(8)
    q = rng.random((40, 5)).astype(np.float32)
    r = rng.random((70, 5)).astype(np.float32)
    np.testing.assert_allclose(ok.kde(q, r, 0.3)[0], ok.kde_numpy(q, r, 0.3), rtol=1e-13)


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(10, 60))
    d = int(rng.integers(1, 4))
    ls = int(rng.integers(1, 6))
    x = rng.random((n, d)).astype(np.float32)
    h = float(rng.uniform(0.05, 0.5))
    eps = float(10.0 ** rng.uniform(-4, 0))
    return x, h, eps, ls


def test_literal_dual_tree_within_eps():
    approximated = 0
    for seed in range(120):
        x, h, eps, ls = _case(seed)
        t = dt.DualTreeKDE(x, x, h, eps, leaf_size=ls)
        f = t.run()
        exact, _ = ok.kde(x, x, h)
        assert np.abs(f - exact).max() <= eps * (1 + 1e-9) + 1e-12, seed
        approximated += t.approximations
    assert approximated > 0


def test_literal_dual_tree_eps_zero_is_exact():
    for seed in range(40):
        x, h, _, ls = _case(seed)
        f = dt.DualTreeKDE(x, x, h, 0.0, leaf_size=ls).run()
        np.testing.assert_allclose(f, ok.kde(x, x, h)[0], rtol=1e-12)


def test_printed_comparison_breaks_the_bound():
    """Algorithm 9 as printed approximates when B_K >= eps / |S_r|: the
    error then exceeds eps on these seeded inputs."""
    worst = 0.0
    for seed in range(60):
        x, h, eps, ls = _case(seed)
        f = dt.DualTreeKDE(x, x, h, eps, leaf_size=ls, printed=True).run()
        worst = max(worst, float(np.abs(f - ok.kde(x, x, h)[0]).max() / eps))
    assert worst > 1.0
