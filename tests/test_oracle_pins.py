"""Pins for the CPU oracle: checks against facts fixed by the paper and by the mathematics.

None of these compare the oracle with itself.  They use

* the textbook definition of mu by trial division (independent prime list
  built here with numpy, not by the oracle),
* hand values M(1..5) = 1, 0, -1, -1, -2 (Section 1 definition),
* the identity sum_{x<=n} M(floor(n/x)) = 1 (Section 2),
* the printed extreme ratio |M(n)|/sqrt(n) = 0.570591 at n = 7766842813
  (Section 1), which fixes |M(7766842813)| uniquely,
* agreement of the two oracle tiers, which share nothing but the O1 table
  at small arguments,
* for the interval tier (Section 6), brute-force extremes of M(n)/sqrt(n)
  with decimal square roots over trial-division mu, and the printed extreme
  above as the extreme of a window around it.

``test_planted_mistakes`` rebuilds the oracle with one plausible mistake at a
time (textual edits of a copy of the C source, compiled in a temp dir) and
requires that some pin fails for every such mutant.
"""
from __future__ import annotations

import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction
import shutil
import subprocess

import numpy as np
import pytest

import oracle


def _primes_np(limit: int) -> np.ndarray:
    s = np.ones(limit + 1, dtype=bool)
    s[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0].astype(np.int64)


_PRIMES = _primes_np(6_000_000)


def mu_trial(y: int) -> int:
    """Textbook mu by trial division (y <= 3.6e13 with the prime list above)."""
    assert y <= int(_PRIMES[-1]) ** 2
    if y == 0:
        return 0
    sign = 1
    for p in _PRIMES:
        p = int(p)
        if p * p > y:
            break
        if y % p == 0:
            y //= p
            if y % p == 0:
                return 0
            sign = -sign
    if y > 1:
        sign = -sign
    return sign


def mu_trial_window(y1: int, count: int) -> np.ndarray:
    """Vectorised trial division over a window (numpy object ints, exact)."""
    ys = [y1 + i for i in range(count)]
    out = np.empty(count, dtype=np.int8)
    lim = math.isqrt(y1 + count) + 1
    assert lim <= int(_PRIMES[-1])
    ps = _PRIMES[_PRIMES <= lim]
    arr = np.array(ys, dtype=np.int64)
    for i, y in enumerate(ys):
        divs = ps[(arr[i] % ps) == 0]
        r = y
        sign = 1
        ok = True
        for p in divs:
            p = int(p)
            r //= p
            if r % p == 0:
                ok = False
                break
            sign = -sign
        if not ok:
            out[i] = 0
            continue
        if r > 1:
            sign = -sign
        out[i] = sign
    return out


# ---------------------------------------------------------------- pin bodies
# Each takes an OracleLib so the planted-mistake test can rerun them.

def pin_mu_textbook(lib):
    mu = lib.mu_range(0, 3000)
    ref = np.array([mu_trial(y) for y in range(3001)], dtype=np.int8)
    assert np.array_equal(mu, ref)


def pin_mu_high_windows(lib):
    for y1 in (10**9 - 500, 2**40 - 300, 10**12 - 250, 999_999_999_989 * 31):
        got = lib.mu_range(y1, y1 + 599)
        assert np.array_equal(got, mu_trial_window(y1, 600)), y1


def pin_small_values(lib):
    assert list(lib.mertens_many([0, 1, 2, 3, 4, 5])) == [0, 1, 0, -1, -1, -2]
    tab = lib.mertens_table(5)
    assert list(tab) == [0, 1, 0, -1, -1, -2]


def _identity_sum(tab: np.ndarray, n: int) -> int:
    """sum_{x=1}^{n} M(floor(n/x)) by runs of equal quotient (plain loops)."""
    s, x = 0, 1
    while x <= n:
        q = n // x
        x2 = n // q
        s += (x2 - x + 1) * int(tab[q])
        x = x2 + 1
    return s


def pin_identity(lib):
    N = 2_000_000
    tab = lib.mertens_table(N)
    rng = np.random.default_rng(7)
    for n in [1, 2, 3, 4, 97, N] + [int(v) for v in rng.integers(2, N, 40)]:
        assert _identity_sum(tab, n) == 1, n


def pin_tiers_agree(lib):
    rng = np.random.default_rng(11)
    ns = [int(v) for v in rng.integers(10**5, 4 * 10**7, 12)] + [4 * 10**7]
    direct = lib.mertens_many(ns)
    tab = lib.mertens_table(20_000)  # T >= sqrt(4e7), far below n: deep recursion
    for n, d in zip(ns, direct):
        assert lib.identity(n, tab)[0] == int(d), n


def pin_byproducts(lib):
    n = 10**7 + 12345
    L = 2500
    tab_full = lib.mertens_table(n)
    _, byp = lib.identity(n, lib.mertens_table(5000), L)
    ref = np.array([tab_full[n // c] for c in range(1, L + 1)], dtype=np.int64)
    assert np.array_equal(byp, ref)


def pin_paper_extreme_ratio(lib):
    # Section 1: the largest known |M(n)|/sqrt(n) is 0.570591, at n = 7766842813.
    n = 7766842813
    m, _ = lib.identity(n, lib.mertens_table(5_000_000))
    assert round(abs(m) / math.sqrt(n), 6) == 0.570591
    # the printed ratio determines |M(n)| uniquely: no other integer rounds to it
    lo = math.ceil((0.5705905) * math.sqrt(n))
    hi = math.floor((0.5705915) * math.sqrt(n))
    assert lo == hi == abs(m)


def _extremes_decimal(ms, ns):
    """(argmin, argmax) of m/sqrt(n) with 50-digit decimal square roots; values
    within 1e-40 of each other count as equal and the smaller n is kept."""
    getcontext().prec = 50
    r = [Decimal(m) / Decimal(n).sqrt() for m, n in zip(ms, ns)]
    eps = Decimal("1e-40")
    lo = hi = 0
    for i in range(1, len(r)):
        if r[i] < r[lo] - eps:
            lo = i
        if r[i] > r[hi] + eps:
            hi = i
    return ns[lo], ns[hi]


_MU_TRIAL_20K = None


def _mertens_trial(N: int) -> list:
    """M(0..N) from textbook trial-division mu (N <= 20000), cached."""
    global _MU_TRIAL_20K
    if _MU_TRIAL_20K is None:
        run, out = 0, [0]
        for y in range(1, 20001):
            run += mu_trial(y)
            out.append(run)
        _MU_TRIAL_20K = out
    return _MU_TRIAL_20K[: N + 1]


def pin_interval_brute(lib):
    # Section 6: values on [a, b] from M(a) and the sieve; extremes by brute force
    M = _mertens_trial(20000)
    rng = np.random.default_rng(5)
    cases = [(1, 1), (1, 10), (1, 20000), (2, 2), (13, 13)]
    for _ in range(30):
        a = int(rng.integers(1, 19000))
        cases.append((a, a + int(rng.integers(0, 1000))))
    # ties: an interval between two zeros of M over which M never rises above
    # zero (largest ratio 0 at both ends), and the same below zero
    zeros = [n for n in range(1, 20001) if M[n] == 0]
    for sgn in (1, -1):
        for z1, z2 in zip(zeros, zeros[1:]):
            if z2 > z1 + 2 and all(sgn * M[n] <= 0 for n in range(z1, z2 + 1)):
                cases.append((z1, z2))
                break
    for a, b in cases:
        got = lib.interval(a, b, M[a])
        ns = list(range(a, b + 1))
        nmin, nmax = _extremes_decimal([M[n] for n in ns], ns)
        assert got["m_b"] == M[b], (a, b)
        assert (got["n_min"], got["m_min"]) == (nmin, M[nmin]), (a, b)
        assert (got["n_max"], got["m_max"]) == (nmax, M[nmax]), (a, b)


def pin_interval_long(lib):
    # an interval across many oracle sub-blocks, against the O1 table and a
    # float filter plus exact integer comparison done here
    a, b = 1_000_003, 3_500_000
    tab = lib.mertens_table(b).astype(np.int64)
    got = lib.interval(a, b, int(tab[a]))
    assert got["m_b"] == int(tab[b])
    ns = np.arange(a, b + 1)
    ms = tab[a:]
    r = ms / np.sqrt(ns.astype(np.float64))
    def order(t):  # sign(m) m^2 / n orders pairs exactly as m / sqrt(n)
        m, n = t
        return ((m > 0) - (m < 0)) * Fraction(m * m, n)

    for key, sgn in (("n_min", 1), ("n_max", -1)):
        best = np.min(sgn * r)
        cand = np.nonzero(np.abs(sgn * r - best) <= 1e-9 * abs(best) + 1e-12)[0]
        pairs = [(int(ms[i]), int(ns[i])) for i in cand]
        want = min(pairs, key=lambda t: (sgn * order(t), t[1]))
        assert got[key] == want[1], key


def pin_interval_paper_extreme(lib):
    # Section 1: |M(n)|/sqrt(n) = 0.570591 at n = 7766842813 is the largest
    # known ratio, so it is the extreme of any window around it
    n0 = 7766842813
    a, b = n0 - 2**16, n0 + 2**16
    tab = lib.mertens_table(5_000_000)
    m_a, _ = lib.identity(a, tab)
    m_b, _ = lib.identity(b, tab)
    got = lib.interval(a, b, m_a)
    assert got["m_b"] == m_b
    far = max((got["n_min"], got["m_min"]), (got["n_max"], got["m_max"]),
              key=lambda t: abs(t[1]) / math.sqrt(t[0]))
    assert far[0] == n0
    assert round(abs(far[1]) / math.sqrt(n0), 6) == 0.570591


ALL_PINS = [pin_mu_textbook, pin_mu_high_windows, pin_small_values, pin_identity,
            pin_tiers_agree, pin_byproducts, pin_paper_extreme_ratio, pin_interval_brute,
            pin_interval_long, pin_interval_paper_extreme]


# ---------------------------------------------------------------- tests

@pytest.fixture(scope="module")
def lib():
    oracle.build()
    return oracle.default()


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, lib):
    pin(lib)


def test_identity_oracle_independent_of_T(lib):
    n = 123_456_789_012
    vals = {lib.identity(n, lib.mertens_table(T))[0] for T in (351_364, 1_000_000, 24_779_000)}
    assert len(vals) == 1


def test_errors(lib):
    with pytest.raises(RuntimeError):
        lib.identity(10**12, lib.mertens_table(1000))  # T below sqrt(n)


MUTANTS = [
    ("square entries not zeroed", "            mag[i] = 0;\n", "            ;\n"),
    ("sign rule swapped", "mag[i] == y ? s : -s", "mag[i] == y ? -s : s"),
    ("sign not toggled per prime", "neg[i] ^= 1;", "neg[i] = 1;"),
    ("sieving primes only to y2^(1/4)", "uint64_t plimit = ceil_sqrt(y2);",
     "uint64_t plimit = isqrt_u64(isqrt_u64(y2)) + 1;"),
    ("identity constant dropped", "uint64_t s = 1;", "uint64_t s = 0;"),
    ("run length off by one quotient", "m / y - m / (y + 1)", "m / y - m / (y + 2)"),
    ("memo index j*x -> x", "s -= big[j * x];", "s -= big[x];"),
    ("first sum bound exclusive", "for (uint64_t x = 2; x <= xmax; x++)",
     "for (uint64_t x = 2; x < xmax; x++)"),
    ("second sum bound short", "for (uint64_t y = 1; y < t; y++)",
     "for (uint64_t y = 1; y + 1 < t; y++)"),
    ("negative ratios ordered like positive ones", "return s1 > 0 ? l < r : l > r;",
     "return l < r;"),
    ("ties keep the later n", "if (ratio_less(mmax, nmax, m, n)) {",
     "if (!ratio_less(m, n, mmax, nmax)) {"),
    ("interval chunk starts one early", "mu_block(c + 1, c2, pr, np, mag, neg, mu);",
     "mu_block(c, c2 - 1, pr, np, mag, neg, mu);"),
    ("squares compared without the other n", "* n2;\n", "* n1;\n"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(name, old, new, tmp_path):
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", so, str(mpath), "-lm"])
    mlib = oracle.OracleLib(so)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(mlib)
        except (AssertionError, RuntimeError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutant: {name}"
