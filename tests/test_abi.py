"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, rejects bad arguments, and its host build of the division routine
is exact (no GPU needed for any of these)."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1108_0135_amd import mertens as mt


def test_exports_every_header_symbol():
    syms = mt.header_symbols()
    assert len(syms) >= 11
    lib = ctypes.CDLL(mt.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s


def test_strerror_codes():
    lib = mt.raw()
    for code in (0, mt.EINVAL, mt.ENOMEM, mt.ENODEV, mt.ERANGE, mt.EIO, mt.EAGAIN,
                 mt.EINPROGRESS):
        assert lib.mertens_strerror(code)
    assert lib.mertens_strerror(-9999) == b"unknown error"


def test_bad_arguments_without_gpu():
    lib = mt.raw()
    # invalid block sizes are rejected before any device call
    for blk in (1, 65536, 131072 + 64, (1 << 31) + 131072):
        assert lib.mertens_init(0, blk) == mt.EINVAL
    # count 0 touches nothing; null pointers with count > 0 are rejected
    assert lib.mertens_query(None, 0, None) == 0
    assert lib.mertens_query(None, 3, None) == mt.EINVAL
    assert lib.mertens_set_param(b"nope", 1.0) == mt.EINVAL
    assert lib.mertens_set_param(b"beta", 0.0) == mt.EINVAL
    assert lib.mertens_set_param(b"ychunk", 100.0) == mt.EINVAL  # not a multiple of 64
    assert lib.mertens_set_param(b"ychunk", float(1 << 21)) == mt.EINVAL  # fp64 sums inexact
    for key, bad in ((b"sieve_ahead", 0.0), (b"sieve_ahead", 257.0), (b"rl_fast", 2.0),
                     (b"update_window", 16.0), (b"update_window", 27.5), (b"kbal", -1.0),
                     (b"kbal", 2.5), (b"klchunk", 256.0), (b"graph", 0.5),
                     (b"bucket_min", 0.0)):
        assert lib.mertens_set_param(key, bad) == mt.EINVAL, key
    # interval: a >= 1, a <= b <= 2^64 - 2^32, values need room and at most 2^28 of them
    vals = np.zeros(4, dtype=np.int64)
    for a, b, cap in ((0, 5, 0), (9, 8, 0), (1, 2**64 - 2**32 + 1, 0), (1, 10, 4),
                      (10**12, 10**12 + 2**28, 2**29)):
        use = cap > 0
        assert lib.mertens_interval(a, b, None, None, None, None,
                                    mt._i64p(vals) if use else None, cap) == mt.EINVAL, (a, b)
    # wide arguments: n_hi < 2^32; wide_bits in 33..64
    lo = np.array([1], dtype=np.uint64)
    hi = np.array([1 << 32], dtype=np.uint64)
    out = np.zeros(1, dtype=np.int64)
    assert lib.mertens_query_wide(mt._u64p(lo), mt._u64p(hi), 1, mt._i64p(out)) == mt.EINVAL
    assert lib.mertens_query_wide(None, None, 0, None) == 0
    for bad in (32.0, 65.0, 40.5):
        assert lib.mertens_set_param(b"wide_bits", bad) == mt.EINVAL, bad
    # divisor outside [1, 2^32)
    n = np.array([5], dtype=np.uint64)
    for bad in (0, 1 << 32):
        d = np.array([bad], dtype=np.uint64)
        q = np.zeros(1, dtype=np.uint64)
        assert lib.mertens_debug_div(mt._u64p(n), mt._u64p(d), 1, mt._u64p(q), 0) == mt.EINVAL


def test_no_device_here_or_initialised():
    # on a host without a GPU, init reports ENODEV and queries refuse to run
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = mt.raw()
    assert lib.mertens_init(0, 0) == mt.ENODEV
    n = np.array([10], dtype=np.uint64)
    out = np.zeros(1, dtype=np.int64)
    assert lib.mertens_query(mt._u64p(n), 1, mt._i64p(out)) == mt.ENODEV
    assert lib.mertens_interval(5, 10, None, None, None, None, None, 0) == mt.ENODEV


def _div_cases(rng):
    ds, ns = [], []
    M64 = (1 << 64) - 1
    # every d <= 2^12 and powers of two / neighbours, at quotient boundaries
    dlist = list(range(1, 4097)) + [2**k + e for k in range(12, 32) for e in (-1, 0, 1)]
    dlist += [int(v) for v in rng.integers(1, 1 << 32, 2000)]
    dlist = [d for d in dlist if 1 <= d < (1 << 32)]
    for d in dlist:
        qs = [int(rng.integers(0, M64 // d + 1, dtype=np.uint64)), M64 // d, 1, 0]
        for q in qs:
            for n in (q * d - 1, q * d, q * d + d - 1):
                if 0 <= n <= M64:
                    ds.append(d)
                    ns.append(n)
        ds.append(d)
        ns.append(M64)
    return np.array(ns, dtype=np.uint64), np.array(ds, dtype=np.uint64)


def test_gm_division_host_exact():
    rng = np.random.default_rng(3)
    n, d = _div_cases(rng)
    q = mt.debug_div(n, d, on_device=False)
    ref = np.array([int(a) // int(b) for a, b in zip(n, d)], dtype=np.uint64)
    assert np.array_equal(q, ref)


def _wide_cases(rng, op: int, count: int = 4000):
    """(m, d) pairs for each routine of mertens_debug_wide, with the edges of
    its range: random bit lengths, d = 1 and the largest d, m = 0, the largest
    m, and m = q d + r with r in {0, 1, d - 1} (quotients that sit exactly on,
    just above and just below an integer boundary)."""
    def rnd(bits):
        b = int(rng.integers(0, bits + 1))
        return int.from_bytes(rng.bytes(16), "little") >> (128 - b) if b else 0
    ms, ds = [], []
    mbits, dbits = {0: (128, 64), 1: (96, 32), 2: (114, 64)}[op]
    for _ in range(count):
        d = max(1, rnd(dbits))
        if op == 2:
            q = rnd(50) if rng.random() < 0.9 else (1 << 50) - 1
            if q * d >= 1 << 128:
                d = max(1, ((1 << 128) - 1) // max(q, 1))
            r = [0, 1, d - 1, rnd(64) % d][int(rng.integers(0, 4))] if d > 1 else 0
            m = q * d + r
        else:
            m = rnd(mbits)
            if rng.random() < 0.3:  # near a multiple of d
                q = m // d
                m = min(q * d + [0, 1, d - 1][int(rng.integers(0, 3))], (1 << mbits) - 1)
        ms.append(m)
        ds.append(d)
    top = (1 << mbits) - 1
    ms += [0, top, top, 1 << 64 if mbits > 64 else 1, top]
    ds += [1, 1, (1 << dbits) - 1, 3, 2] if op != 2 else [1, 1 << 20, 1 << 63, 3, 1 << 62]
    if op == 2:  # keep every quotient below 2^50
        ms[-4:] = [(1 << 70) - 1, (1 << 113) - 1, 5, (1 << 111) + 7]
    return ms, ds


def _wide_expect(op, ms, ds):
    return [m // d if op != 1 else (m // d) % (1 << 64) for m, d in zip(ms, ds)]


@pytest.mark.parametrize("op", [0, 1, 2])
def test_wide_division_host(op):
    # host build of the 128-bit quotient routines against Python integers
    rng = np.random.default_rng(30 + op)
    ms, ds = _wide_cases(rng, op)
    assert mt.debug_wide(ms, ds, op, on_device=False) == _wide_expect(op, ms, ds)


def test_wide_division_ranges():
    lib = mt.raw()
    one = np.array([1], dtype=np.uint64)
    zero = np.array([0], dtype=np.uint64)
    big = np.array([1 << 32], dtype=np.uint64)
    q = np.zeros(1, dtype=np.uint64)
    q2 = np.zeros(1, dtype=np.uint64)
    f = lambda lo, hi, d, op: lib.mertens_debug_wide(mt._u64p(lo), mt._u64p(hi), mt._u64p(d), 1,
                                                     mt._u64p(q), mt._u64p(q2), op, 0)
    assert f(one, zero, zero, 0) == mt.EINVAL      # d = 0
    assert f(one, zero, big, 1) == mt.EINVAL       # digit steps need d < 2^32
    assert f(one, big, one, 1) == mt.EINVAL        # ... and m < 2^96
    assert f(one, one, one, 2) == mt.EINVAL        # quotient 2^64 + 1 >= 2^50
    assert f(one, zero, one, 3) == mt.EINVAL       # no such op
    out = ctypes.c_uint64(0)
    assert lib.mertens_debug_runsum(5, 1 << 18, 10, ctypes.byref(out)) == mt.EINVAL  # n >= 2^82
    assert lib.mertens_debug_runsum(5, 0, 0, ctypes.byref(out)) == mt.EINVAL         # L = 0
    assert lib.mertens_debug_runsum(5, 0, 10, ctypes.byref(out)) == mt.EINVAL        # n/(L+1) = 0


def test_host_prime_table():
    # the sieving primes (5 <= p <= limit) of the host table against prime
    # counts: pi(10^6) = 78498, pi(10^9) = 50847534, pi(2^32) = 203280221, and
    # against a direct numpy sieve on small limits (count, largest, sum)
    for limit in (4, 5, 6, 1000, 2**19, 2**20 + 3, 10**6):
        s = np.ones(limit + 1, dtype=bool)
        s[:2] = False
        for i in range(2, int(limit ** 0.5) + 1):
            if s[i]:
                s[i * i::i] = False
        ps = np.nonzero(s)[0]
        ps = ps[ps >= 5]
        want = (len(ps), int(ps[-1]) if len(ps) else 0, int(ps.sum()))
        assert mt.debug_primes(limit) == want, limit
    assert mt.debug_primes(10**9)[0] == 50847534 - 2
    count, last, _ = mt.debug_primes(2**32)
    assert (count, last) == (203280221 - 2, 4294967291)
    lib = mt.raw()
    c = ctypes.c_uint64(0)
    assert lib.mertens_debug_primes(2**32 + 1, ctypes.byref(c), ctypes.byref(c),
                                    ctypes.byref(c)) == mt.EINVAL
