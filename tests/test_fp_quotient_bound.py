"""The fp64 quotient rule of the run-length update, checked on the CPU.

For m < 2^48 and 1 <= y < 2^32, the device takes floor(m/y) as
floor(RN(m * r')) with r' = (1/y)(1 + b), b in [2^-50.2, 2^-49.8]: a
hardware estimate refined by one Newton step, then a second step aimed at
(1 + 2^-50)/y (no remainder test).  The construction of r' is checked in
exact rational arithmetic (test_biased_newton_step); the rule is checked
with r' = RN(1/y) raised by three, four and five units in the last place,
biases of 2^-51.4 ... 2^-49.7 that cover b's range.  IEEE binary64 multiply
and divide are correctly rounded on the CPU as on the GPU, so numpy
reproduces the rule's values bit for bit.  It must hold on random pairs and
on the adversarial ones: exact multiples (m = k y), m = k y - 1 just below
them, and the largest m allowed.
"""
from fractions import Fraction
import math

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


# The reciprocal itself: r1 = (1 - e1)/k after the first Newton step (the
# hardware estimate's error squared, near 2^-40 or far below), then
# e = RN(1 + 2^-50 - k r1) (one fused rounding) and r' = RN(r1 + r1 e).

def _biased_newton(k, r1):
    one_c = Fraction(1) + Fraction(1, 2**50)
    assert float(one_c) == 1.0 + 2.0**-50  # exactly representable
    e = float(one_c - k * Fraction(r1))
    return float(Fraction(r1) + Fraction(r1) * Fraction(e))


def _bias_log2(k, r):
    b = Fraction(r) * k - 1
    assert b > 0
    return math.log2(b)


def test_biased_newton_step():
    rng = np.random.default_rng(15)
    ks = [1, 2, 3, 5, 7, 2**20 - 1, 2**20, 2**20 + 1, 2**31 - 1, 2**31, 2**32 - 1,
          2**32 - 5, 3 * 2**29, 1431655765]
    ks += [int(v) for v in rng.integers(1, 2**32, 3000)]
    lo, hi = 0.0, -100.0
    for k in ks:
        rn = 1.0 / k
        base = [rn, float(np.nextafter(rn, 0.0)), float(np.nextafter(rn, 1.0))]
        for eps in (2.0**-40, -2.0**-40, 2.0**-45, -2.0**-45):
            base.append(float(Fraction(1, k) * (1 + Fraction(eps))))
        for r1 in base:
            t = _bias_log2(k, _biased_newton(k, r1))
            assert -50.2 <= t <= -49.8, (k, r1, t)
            lo, hi = min(lo, t), max(hi, t)
    assert lo < -50.1 and hi > -49.9  # both ends of the range are reached


def test_biased_reciprocal_floors():
    # the floor rules with r' built as on the device (r1 = RN(1/k) and one
    # unit off), on the adversarial m of each kind
    rng = np.random.default_rng(16)
    bad = []
    for _ in range(1500):
        k = int(rng.integers(1, 2**32))
        rn = 1.0 / k
        for r1 in (rn, float(np.nextafter(rn, 0.0)), float(np.nextafter(rn, 1.0))):
            ru = _biased_newton(k, r1)
            num, den = Fraction(ru).as_integer_ratio()
            qmax = (2**48 - 1) // k
            if qmax < 1:
                continue
            q = int(rng.integers(1, qmax + 1))
            for m in (q * k, q * k + k - 1, q * k - 1):
                if not 0 < m < 2**48:
                    continue
                # plain product: floor(RN(m r'))
                if math.floor(float(Fraction(m * num, den))) != m // k:
                    bad.append(("plain", m, k, r1))
                # the magic-constant low word, for quotients below 2^23
                if m // k < 2**23:
                    v = float(Fraction(2 * m * num + (2**53 - 1) * den, 2 * den))
                    low = int(np.array([v]).view(np.int64)[0]) - \
                        int(np.array([2.0**52]).view(np.int64)[0])
                    if low != m // k:
                        bad.append(("magic", m, k, r1))
                # the fused block offset, for a block [y1, y2] holding q with
                # y2 - y1 < y1
                y1 = (m // k) // 2 + 1 if m // k >= 2 else 0
                if y1 == 0 or m // k - y1 < y1:
                    off = int(float(Fraction(m * num - y1 * den, den)))
                    if off != m // k - y1:
                        bad.append(("fused", m, k, r1, y1))
    assert not bad, bad[:5]
