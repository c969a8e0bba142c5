"""The fp64 quotient rule of the run-length update, checked on the CPU.

For m < 2^48 and 1 <= y < 2^32, the device takes floor(m/y) as
floor(RN(m * r')) with r' a reciprocal r of y within one unit in the last
place (a hardware estimate refined by two Newton steps) raised by four
units in the last place (no remainder test).  The rule is checked here with
r = RN(1/y) and with r one unit below and above it (a wider error than the
device's): IEEE binary64 multiply and divide are correctly rounded on the
CPU as on the GPU, so numpy reproduces the rule's values bit for bit.  It
must hold on random pairs and on the adversarial ones: exact multiples
(m = k y), m = k y - 1 just below them, and the largest m allowed.
"""
import numpy as np


def _floor_quot(m, y, err_units=0):
    r = 1.0 / y.astype(np.float64)
    ru = (r.view(np.int64) + 4 + err_units).view(np.float64)
    return np.floor(m.astype(np.float64) * ru).astype(np.uint64)


def _all_errors(m, y):
    return all(np.array_equal(_floor_quot(m, y, e), m // y) for e in (-1, 0, 1))


def test_random_pairs():
    rng = np.random.default_rng(11)
    for hi_bits in (20, 32, 40, 46, 48):
        m = rng.integers(1, 2**hi_bits, 200_000, dtype=np.uint64)
        y = rng.integers(1, 2**32, 200_000, dtype=np.uint64)
        y = np.minimum(y, m)  # quotients >= 1, as in the sweep
        assert _all_errors(m, y)


def test_exact_multiples_and_neighbours():
    rng = np.random.default_rng(12)
    y = rng.integers(2, 2**32, 300_000, dtype=np.uint64)
    kmax = (np.uint64(2**48 - 2) // y).astype(np.uint64)
    k = (rng.random(y.size) * kmax.astype(np.float64)).astype(np.uint64) + np.uint64(1)
    k = np.minimum(k, kmax)
    m = k * y
    ok = (m < np.uint64(2**48)) & (k >= 1)
    m, y = m[ok], y[ok]
    assert _all_errors(m, y)
    assert _all_errors(m - np.uint64(1), y)
    assert _all_errors(m + np.uint64(1), y)


def test_largest_m_small_y():
    m = np.full(4096, 2**48 - 1, dtype=np.uint64) - np.arange(4096, dtype=np.uint64)
    for y0 in (1, 2, 3, 7, 65536, 2**31 - 1):
        y = np.full(m.size, y0, dtype=np.uint64)
        assert _all_errors(m, y)
