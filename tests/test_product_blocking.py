"""The library's blocking analysis (host code, no device work), pinned on its
own against series with a known variance of the mean, and compared with the
oracle's separately written routine on the same series."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F


def _ar1(phi, n, seed, burn=1000):
    rng = np.random.default_rng(seed)
    eps = rng.normal(size=n + burn)
    x = np.zeros_like(eps)
    for t in range(1, len(eps)):
        x[t] = phi * x[t - 1] + eps[t]
    return x[burn:]


def test_ar1_variance_of_the_mean():
    n, phi = 1 << 16, 0.8
    x = 5.0 + _ar1(phi, n, 3)
    mean, err = F.fciqmc_blocking(x)
    assert abs(mean - x.mean()) < 1e-12
    exact = math.sqrt(1.0 / (1 - phi) ** 2 / n)
    assert abs(err - exact) / exact < 0.15


def test_uncorrelated_ratio_follows_error_propagation():
    n = 1 << 15
    rng = np.random.default_rng(5)
    num = 3.0 + 0.1 * rng.normal(size=n)
    den = 2.0 + 0.05 * rng.normal(size=n)
    r, err = F.fciqmc_blocking(num, den)
    assert abs(r - num.mean() / den.mean()) < 1e-12
    exact = (3 / 2) * math.sqrt((0.1 / 3) ** 2 + (0.05 / 2) ** 2) / math.sqrt(n)
    assert abs(err - exact) / exact < 0.15


def test_fully_correlated_ratio_has_no_error():
    """num = 2.5 den exactly: the ratio is constant, its error zero to rounding."""
    den = 10.0 + _ar1(0.5, 4096, 9)
    r, err = F.fciqmc_blocking(2.5 * den, den)
    assert abs(r - 2.5) < 1e-13 and err < 1e-9


def test_short_series_has_no_error_bar():
    m, e = F.fciqmc_blocking(np.arange(10.0))
    assert m == 4.5 and math.isnan(e)


@pytest.mark.parametrize("seed,n,phi", [(1, 700, 0.9), (2, 5000, 0.6), (3, 1 << 14, 0.95),
                                        (4, 12345, 0.3)])
def test_agrees_with_oracle(seed, n, phi):
    """Correlated (num, C_0)-like series with a drift at the start: the same mean
    and error bar as the oracle's two-pass routine to 1e-10 relative."""
    rng = np.random.default_rng(seed)
    den = 1000.0 + 50.0 * _ar1(phi, n, seed) + np.linspace(-300, 0, n) * (np.arange(n) < n // 5)
    num = -0.7 * den + 20.0 * _ar1(phi, n, seed + 100) + rng.normal(size=n)
    for d in (den, None):
        mp, ep = F.fciqmc_blocking(num, d)
        mo, eo, lvl = O.blocking(num, d)
        assert lvl >= 0
        assert abs(mp - mo) <= 1e-12 * abs(mo)
        assert abs(ep - eo) <= 1e-10 * eo, (ep, eo)
