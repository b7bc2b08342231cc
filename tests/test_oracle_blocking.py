"""Pin for the blocking analysis: an AR(1) series has a known variance of the mean."""
import math

import numpy as np

from oracle import oracle as O


def _ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    eps = rng.normal(size=n + 1000)
    x = np.zeros_like(eps)
    for t in range(1, len(eps)):
        x[t] = phi * x[t - 1] + eps[t]
    return x[1000:]


def test_blocking_ar1_single_series():
    n, phi = 1 << 16, 0.8
    x = 5.0 + _ar1(phi, n, 3)
    exact = math.sqrt(1.0 / (1 - phi) ** 2 / n)
    mean, err, lvl = O.blocking(x)
    assert abs(mean - x.mean()) < 1e-12
    assert lvl > 0
    assert abs(err - exact) / exact < 0.15


def test_blocking_uncorrelated():
    n = 1 << 15
    x = np.random.default_rng(4).normal(size=n) + 2.0
    mean, err, lvl = O.blocking(x)
    assert abs(err - 1 / math.sqrt(n)) / (1 / math.sqrt(n)) < 0.15


def test_blocking_ratio_matches_delta_method():
    # With independent (num, den) the ratio error follows first-order propagation.
    n = 1 << 15
    rng = np.random.default_rng(5)
    num = 3.0 + 0.1 * rng.normal(size=n)
    den = 2.0 + 0.05 * rng.normal(size=n)
    r, err, lvl = O.blocking(num, den)
    assert abs(r - num.mean() / den.mean()) < 1e-12
    exact = (3 / 2) * math.sqrt((0.1 / 3) ** 2 + (0.05 / 2) ** 2) / math.sqrt(n)
    assert abs(err - exact) / exact < 0.15


def test_blocking_short_series_has_no_error_bar():
    mean, err, lvl = O.blocking(np.arange(10.0))
    assert math.isnan(err) and lvl == -1
