"""CPU model of the split the GPU kernels use, checked against the oracle.

The device path splits S[x] = sum_{k=k0}^{m} M(floor(m/k)) at
K = max(k0-1, floor(beta*sqrt(m)), floor(m/2^32)), Y = floor(m/(K+1)):

    S[x] = sum_{k=k0}^{K} M(floor(m/k)) + sum_{y=1}^{Y} floor(m/y) mu(y) - K M(Y)

(the run-length sum of Section 2 summed by parts), and distributes every
term to the y-block that holds its argument.  This test re-derives that
bookkeeping in plain numpy on small n, for several u, block lengths and
beta, and checks the resulting A[x] = M(floor(n/x)) against the oracle.
It pins the formulas the kernels implement before any GPU run, including the
split of the 128-bit entries (K >= floor(m / 2^32), run-length quotients
mod 2^64 by 32-bit digit steps), modelled with narrower digits.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle


def model(n: int, u: int, B: int, beta: float, mu: np.ndarray, M: np.ndarray,
          shift: int = 32, quot=None) -> np.ndarray:
    L = max(1, n // u)
    ymax = n // (L + 1)
    S = np.zeros(L + 1, dtype=object)
    meta = []
    for x in range(1, L + 1):
        m = n // x
        k0 = L // x + 1
        K = max(k0 - 1, int(beta * math.isqrt(m)), m >> shift)
        Y = m // (K + 1)
        meta.append((m, k0, K, Y))
    order = list(range(ymax // B + 1))
    order.reverse()  # block order must not matter (sums commute)
    for bi in order:
        y1, y2 = bi * B, min(bi * B + B - 1, ymax)
        y1e = max(y1, 1)
        for x, (m, k0, K, Y) in enumerate(meta, start=1):
            klo = max(k0, m // (y2 + 1) + 1)
            khi = min(K, m // y1e)
            acc = 0
            for k in range(klo, khi + 1):
                acc += int(M[m // k])
            if y1e <= Y <= y2:
                acc -= K * int(M[Y])
            hi = min(y2, Y)
            if hi >= y1e and quot is None:
                ys = np.arange(y1e, hi + 1, dtype=np.int64)
                acc += int(np.sum((m // ys) * mu[y1e:hi + 1].astype(np.int64)))
            elif hi >= y1e:
                for y in range(y1e, hi + 1):
                    acc += quot(m, y) * int(mu[y])
            S[x] += acc
    A = [0] * (L + 1)
    for x in range(L, 0, -1):
        s = 1 - S[x]
        for k in range(2, L // x + 1):
            s -= A[k * x]
        A[x] = s
    return np.array(A[1:], dtype=np.int64)


@pytest.mark.parametrize("n,u,B,beta", [
    (10**6, 10**4, 64, 1.0),
    (10**6, 10**4, 4096, 0.5),
    (999_983, 5000, 128, 0.3),
    (1_234_567, 11_000, 1 << 16, 0.75),
    (2 * 10**6, 15_874, 1 << 10, 0.5),
    (97, 5, 64, 0.5),
    (2, 2, 64, 0.5),
    (1, 2, 64, 0.5),
    (12, 100, 64, 1.0),
])
def test_model_matches_oracle(n, u, B, beta):
    N = n
    mu = oracle.mu_range(0, N)
    M = oracle.mertens_table(N)
    A = model(n, u, B, beta, mu, M)
    L = max(1, n // u)
    ref = np.array([M[n // c] for c in range(1, L + 1)], dtype=np.int64)
    assert np.array_equal(A, ref)


def digit_quot_low(m: int, y: int, w: int, dbits: int) -> int:
    """floor(m/y) mod 2^w by three dbits-bit digit steps (m < 2^(3 dbits),
    y < 2^dbits), the scheme the 128-bit entries use with dbits = 32, w = 64:
    each step divides (remainder, next digit) by y, and the top digit's
    quotient (a multiple of 2^w) is dropped."""
    mask = (1 << dbits) - 1
    d2, d1, d0 = m >> (2 * dbits), (m >> dbits) & mask, m & mask
    r = d2 % y
    a1 = (r << dbits) | d1
    q1, r = divmod(a1, y)
    a0 = (r << dbits) | d0
    q0 = a0 // y
    return ((q1 << dbits) + q0) % (1 << w)


@pytest.mark.parametrize("n,u,B,shift", [
    (10**6, 10**4, 64, 6),       # K = m >> 6 dominates: long explicit-k ranges, Y < 64
    (2 * 10**6, 15_874, 1024, 8),
    (999_983, 5000, 128, 10),
])
def test_model_wide_split_matches_oracle(n, u, B, shift):
    # the split of the 128-bit entries, K >= floor(m / 2^shift) so Y < 2^shift,
    # with run-length quotients taken mod 2^(2 shift) by digit steps: the
    # dropped multiples of 2^(2 shift) vanish from S mod 2^(2 shift), and the
    # final values are small
    mu = oracle.mu_range(0, n)
    M = oracle.mertens_table(n)
    w = 2 * shift
    A = model(n, u, B, 0.5, mu, M, shift=shift,
              quot=lambda m, y: digit_quot_low(m, y, w, shift))
    L = max(1, n // u)
    ref = np.array([M[n // c] for c in range(1, L + 1)], dtype=np.int64)
    # S is exact only mod 2^w here, and so is A; the true values are below 2^(w-1)
    half = 1 << (w - 1)
    got = np.array([((int(a) + half) % (1 << w)) - half for a in A], dtype=np.int64)
    assert np.array_equal(got, ref)


def test_digit_quot_low_exact():
    rng = np.random.default_rng(3)
    for dbits in (8, 16, 32):
        for _ in range(3000):
            y = int(rng.integers(1, 1 << dbits))
            m = int.from_bytes(rng.bytes(12), "little") >> (96 - 3 * dbits)
            assert digit_quot_low(m, y, 2 * dbits, dbits) == (m // y) % (1 << (2 * dbits))
