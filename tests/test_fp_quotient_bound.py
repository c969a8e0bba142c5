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
from fractions import Fraction

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


# The explicit-k walk folds the block start y1 into one fused multiply-add:
# y - y1 = trunc(RN(m * r' - y1)), with one rounding of the exact value.  It
# is taken for m < 2^48 in a block [y1, y2] with y1 = 0 or y2 - y1 < y1, for
# k with floor(m/k) in the block.  The exact value is formed here in rational
# arithmetic and rounded once (Python's int / int division rounds correctly).

def _fused_off(m, k, y1, err_units):
    r = 1.0 / float(k)
    ru = (np.array([r]).view(np.int64) + 4 + err_units).view(np.float64)[0]
    num, den = Fraction(ru).as_integer_ratio()
    v = (m * num - y1 * den) / den  # correctly rounded
    return int(v)


def _check_block(rng, y1, B, count):
    y2 = y1 + B - 1
    bad = []
    for _ in range(count):
        q = int(rng.integers(y1, y2 + 1))
        if q == 0:
            q = 1
        kmax = (2**48 - 1) // (q + 1)
        if kmax < 1:
            continue
        k = int(rng.integers(max(1, kmax - 1000), kmax + 1)) if rng.random() < 0.5 \
            else int(rng.integers(1, kmax + 1))
        # largest fraction (m = q k + k - 1), exact multiple, and in between
        for m in (q * k + k - 1, q * k, q * k + int(rng.integers(0, k))):
            if m >= 2**48 or not (y1 <= m // k <= y2):
                continue
            for e in (-1, 0, 1):
                if _fused_off(m, k, y1, e) != m // k - y1:
                    bad.append((m, k, y1, e))
    return bad


def test_fused_block_offset():
    rng = np.random.default_rng(13)
    bad = []
    for B in (2**17, 2**24, 2**30, 2**31):
        for b in (0, 1, 2, 3, 7, 1000, 2**20):
            y1 = b * B
            if y1 + B > 2**48:
                continue
            bad += _check_block(rng, y1, B, 600)
    assert not bad, bad[:5]


def test_fused_block_offset_top_of_block():
    # quotients at the top of the block (the largest fused result) with the
    # largest k that reaches them
    bad = []
    for B in (2**30, 2**31):
        for b in (1, 2, 5, 100):
            y1 = b * B
            for q in (y1 + B - 1, y1 + B - 2, y1 + B // 2):
                k = (2**48 - 1) // (q + 1)
                for m in (q * k + k - 1, q * k):
                    for e in (-1, 0, 1):
                        if _fused_off(m, k, y1, e) != m // k - y1:
                            bad.append((m, k, y1, e))
    assert not bad, bad[:5]


# Run-length pairs whose quotients are all below 2^23 take the quotient as
# the low word of fma(m, r', 2^52 - 1/2): the exact value m r' + 2^52 - 1/2
# lies strictly between 2^52 + q - 1/2 and 2^52 + q + 1/2 (q = floor(m/y)),
# so its one rounding to the integer grid of [2^52, 2^53) is 2^52 + q.

MAGIC = 2.0**52 - 0.5


def _magic_quot(m, y, err_units):
    r = 1.0 / float(y)
    ru = (np.array([r]).view(np.int64) + 4 + err_units).view(np.float64)[0]
    assert Fraction(MAGIC) == Fraction(2**53 - 1, 2)  # exactly representable
    num, den = Fraction(ru).as_integer_ratio()
    v = (2 * m * num + (2**53 - 1) * den) / (2 * den)  # correctly rounded
    bits = int(np.array([v]).view(np.int64)[0])
    return bits - int(np.array([2.0**52]).view(np.int64)[0])


def test_magic_low_word():
    rng = np.random.default_rng(14)
    bad = []
    for _ in range(4000):
        m = int(rng.integers(1, 2**48))
        ylo = max(1, m // (2**23 - 1) + 1)  # quotients below 2^23
        if ylo >= 2**32:
            continue
        y = int(rng.integers(ylo, min(2**32, m + 1))) if ylo <= m else ylo
        for mm in (m, (m // y) * y, (m // y) * y + y - 1):
            if mm >= 2**48 or mm < y:
                continue
            for e in (-1, 0, 1):
                if _magic_quot(mm, y, e) != mm // y:
                    bad.append((mm, y, e))
    assert not bad, bad[:5]
