"""Seeded synthetic query sets (shared by the tests, the benchmark and the oracle checks).

This module only draws arguments n; it holds none of the method's arithmetic,
so both the GPU path and the CPU oracle can be fed from it.  Every generator
takes an explicit seed and returns uint64 arrays (n may exceed 2^63).
"""
from __future__ import annotations

import numpy as np

# Powers of ten whose M(n) Table 1 of the paper prints (10^20..10^22 exceed 2^64).
TABLE1 = {
    10**16: -3195437,
    10**17: -21830254,
    10**18: -46758740,
    10**19: 899990187,
    10**20: 461113106,
    10**21: 3395895277,
    10**22: -2061910120,
}
# Section 6: the new extreme value, M(11609864264058592345) = -1,995,900,927.
EXTREME_N = 11609864264058592345
EXTREME_M = -1995900927


def uniform_small(seed: int = 0, count: int = 32, lo: int = 2, hi: int = 10**9) -> np.ndarray:
    """count values of n uniform in [lo, hi] (the brute-force-checkable set)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, count, endpoint=True, dtype=np.uint64)


def log_uniform(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    """count values floor(exp(U(ln lo, ln hi))), as uint64."""
    rng = np.random.default_rng(seed)
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), count))
    return np.array([int(v) for v in x], dtype=np.uint64)


def batch_log_uniform(seed: int = 0, count: int = 256, lo: float = 1e13, hi: float = 1e17) -> np.ndarray:
    """The batched workload: count n log-uniform in [lo, hi]."""
    return log_uniform(seed, count, lo, hi)


def dense_window(seed: int = 0, count: int = 1024, step: int = 997,
                 lo: int = 10**18, hi: int = 18 * 10**18) -> np.ndarray:
    """n_i = n0 + step*i with n0 uniform in [lo, hi] (all below 2^64)."""
    rng = np.random.default_rng(seed)
    n0 = int(rng.integers(lo, hi, endpoint=True, dtype=np.uint64))
    return np.array([n0 + step * i for i in range(count)], dtype=np.uint64)


def poisson_trace(seed: int, rate: float, count: int, lo: float = 1e10, hi: float = 1e18):
    """Arrival times (s, from 0) of a Poisson stream at `rate` q/s, and their n."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    times = np.cumsum(gaps) - gaps[0]
    return times, log_uniform(seed + 1, count, lo, hi)


def interval_around(seed: int, lo: int, hi: int, before: int, after: int):
    """(a, b) = (c - before, c + after) with c uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    c = int(rng.integers(lo, hi, endpoint=True, dtype=np.uint64))
    return c - before, c + after


def extreme_window(before: int = 2**20 + 12345, after: int = 2**20 + 777):
    """(a, b) around the Section 6 extreme (the localization workload)."""
    return EXTREME_N - before, EXTREME_N + after
