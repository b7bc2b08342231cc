"""Pins for the oracle's random-number generator and shift logarithm."""
import ctypes
import math
import os

import numpy as np

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_bits_uniform():
    # Every output bit of consecutive counters is a fair coin (4.5 sigma).
    n = 20000
    bits = np.zeros(128)
    for c in range(n):
        w = O.philox4x32_10([c, 7, 0, 3], [12345, 678])
        for j in range(4):
            x = int(w[j])
            for b in range(32):
                bits[32 * j + b] += (x >> b) & 1
    z = (bits - n / 2) / math.sqrt(n / 4)
    assert np.all(np.abs(z) < 4.5)


def test_log_matches_libm():
    L = O.lib()
    L.orc_log.restype = ctypes.c_double
    L.orc_log.argtypes = [ctypes.c_double]
    rng = np.random.default_rng(1)
    xs = np.concatenate([np.exp(rng.uniform(-40, 40, 20000)), 1 + rng.uniform(-1e-6, 1e-6, 1000),
                         [1.0, 2.0, 0.5, 1e-300, 1e300]])
    for x in xs:
        ref = math.log(x)
        got = L.orc_log(float(x))
        assert abs(got - ref) <= 6e-16 * max(abs(ref), 1e-300) + 1e-300 or abs(got - ref) < 1e-22
    assert L.orc_log(1.0) == 0.0
