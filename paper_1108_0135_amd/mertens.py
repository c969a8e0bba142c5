"""Thin ctypes binding of libmertens.so (the C ABI in include/mertens.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  There is no fallback; if the library is missing
the import of this module raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmertens.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "mertens.h")

EINVAL, ENOMEM, ENODEV, ERANGE, EIO, EAGAIN, EINPROGRESS = -22, -12, -19, -34, -5, -11, -115

STAT_NAMES = ["sieved_y", "blocks", "u", "sum_L", "sum_Y", "sum_k", "ms_sieve",
              "ms_scan", "ms_prep", "ms_update", "ms_finalize", "ms_total", "update_launches",
              "sieve_launches", "rl_quotients", "k_quotients", "bucket_entries", "ms_bucket_fill",
              "bucket_prime_visits", "ms_bucket_regroup", "ms_band", "band_quotients"]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1108_0135_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_u64, _i64, _sz = ctypes.c_uint64, ctypes.c_int64, ctypes.c_size_t
_P = ctypes.POINTER
_sig = {
    "mertens_init": ([_u64, _u64], ctypes.c_int),
    "mertens_query": ([_P(_u64), _sz, _P(_i64)], ctypes.c_int),
    "mertens_query_noalloc": ([_P(_u64), _sz, _P(_i64)], ctypes.c_int),
    "mertens_byproducts": ([_sz, _P(_i64), _sz, _P(_sz)], ctypes.c_int),
    "mertens_query_wide": ([_P(_u64), _P(_u64), _sz, _P(_i64)], ctypes.c_int),
    "mertens_set_stream": ([ctypes.c_void_p], ctypes.c_int),
    "mertens_set_param": ([ctypes.c_char_p, ctypes.c_double], ctypes.c_int),
    "mertens_get_param": ([ctypes.c_char_p, _P(ctypes.c_double)], ctypes.c_int),
    "mertens_stats": ([_P(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "mertens_shutdown": ([], None),
    "mertens_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "mertens_last_error": ([], ctypes.c_char_p),
    "mertens_submit": ([_u64, _P(_u64)], ctypes.c_int),
    "mertens_poll": ([_u64, _P(_i64), _P(ctypes.c_double)], ctypes.c_int),
    "mertens_interval": ([_u64, _u64, _P(_i64), _P(_i64), _P(_u64), _P(_i64), _P(_i64), _sz],
                         ctypes.c_int),
    "mertens_debug_div": ([_P(_u64), _P(_u64), _sz, _P(_u64), ctypes.c_int], ctypes.c_int),
    "mertens_debug_mu": ([_u64, _sz, _P(ctypes.c_int8), _P(_i64)], ctypes.c_int),
    "mertens_debug_runsum": ([_u64, _u64, _u64, _P(_u64)], ctypes.c_int),
    "mertens_debug_primes": ([_u64, _P(_u64), _P(_u64), _P(_u64)], ctypes.c_int),
    "mertens_debug_wide": ([_P(_u64), _P(_u64), _P(_u64), _sz, _P(_u64), _P(_u64), ctypes.c_int,
                            ctypes.c_int], ctypes.c_int),
}
for _name, (_args, _ret) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _ret


class MertensError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.mertens_strerror(code).decode()
        detail = _lib.mertens_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}); {detail}")


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise MertensError(rc, where)


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(_P(_u64))


def _i64p(a: np.ndarray):
    return a.ctypes.data_as(_P(_i64))


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(mertens_\w+)\s*\(", text, re.M)))


def init(u: int = 0, block: int = 0) -> None:
    _check(_lib.mertens_init(u, block), "mertens_init")


def shutdown() -> None:
    _lib.mertens_shutdown()


def query(ns) -> np.ndarray:
    """Exact M(n) for every n (uint64-representable), one shared sweep."""
    arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64).reshape(-1))
    out = np.zeros(arr.size, dtype=np.int64)
    _check(_lib.mertens_query(_u64p(arr), arr.size, _i64p(out)), "mertens_query")
    return out


def query_noalloc(ns) -> np.ndarray:
    """M(n) like query(), through the entry point that allocates no device memory."""
    arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64).reshape(-1))
    out = np.zeros(arr.size, dtype=np.int64)
    _check(_lib.mertens_query_noalloc(_u64p(arr), arr.size, _i64p(out)), "mertens_query_noalloc")
    return out


def query_wide(ns) -> np.ndarray:
    """Exact M(n) for Python ints 0 <= n < 2^96 (words split here, one shared sweep)."""
    ns = [int(v) for v in ns]
    lo = np.array([v & (2**64 - 1) for v in ns], dtype=np.uint64)
    hi = np.array([v >> 64 for v in ns], dtype=np.uint64)
    out = np.zeros(len(ns), dtype=np.int64)
    _check(_lib.mertens_query_wide(_u64p(lo), _u64p(hi), len(ns), _i64p(out)),
           "mertens_query_wide")
    return out


def byproducts(i: int, cap: int | None = None) -> np.ndarray:
    """[M(floor(n_i/c)) for c = 1..L] of query i of the last call."""
    n = _sz(0)
    if cap is None:
        _check(_lib.mertens_byproducts(i, None, 0, ctypes.byref(n)), "mertens_byproducts")
        cap = n.value
    buf = np.zeros(max(cap, 1), dtype=np.int64)
    _check(_lib.mertens_byproducts(i, _i64p(buf), cap, ctypes.byref(n)), "mertens_byproducts")
    return buf[: min(cap, n.value)]


def submit(n: int):
    """Queue M(n) on the serving sweep; returns a ticket, or None if no slot is free."""
    t = _u64(0)
    rc = _lib.mertens_submit(n, ctypes.byref(t))
    if rc == EAGAIN:
        return None
    _check(rc, "mertens_submit")
    return t.value


def poll(ticket: int):
    """(M(n), latency_s) once done, else None."""
    out = _i64(0)
    lat = ctypes.c_double(0.0)
    rc = _lib.mertens_poll(ticket, ctypes.byref(out), ctypes.byref(lat))
    if rc == EINPROGRESS:
        return None
    _check(rc, "mertens_poll")
    return out.value, lat.value


def interval(a: int, b: int, m_a: int | None = None, values: bool = False) -> dict:
    """M over [a, b] from M(a) (computed first when not given): M(b), the n with
    the smallest and largest M(n)/sqrt(n) and M there, and, if asked, every M(n)."""
    ma = _i64(0 if m_a is None else int(m_a))
    mb = _i64(0)
    n_ext = (_u64 * 2)()
    m_ext = (_i64 * 2)()
    vals = np.zeros(b - a + 1 if values else 1, dtype=np.int64)
    _check(_lib.mertens_interval(a, b, None if m_a is None else ctypes.byref(ma), ctypes.byref(mb),
                                 n_ext, m_ext, _i64p(vals) if values else None,
                                 vals.size if values else 0), "mertens_interval")
    out = {"m_b": int(mb.value), "n_min": int(n_ext[0]), "m_min": int(m_ext[0]),
           "n_max": int(n_ext[1]), "m_max": int(m_ext[1])}
    if values:
        out["values"] = vals
    return out


def set_param(key: str, value: float) -> None:
    _check(_lib.mertens_set_param(key.encode(), float(value)), f"mertens_set_param({key})")


TUNING_KEYS = ["tuned", "u_scale", "beta", "ychunk", "kchunk", "kbal", "waves_per_cu", "graph",
               "block_auto", "sieve_ahead", "update_window", "bucket_min", "rl_fast", "wide_bits",
               "band_lo", "band_hi"]


def get_param(key: str) -> float:
    v = ctypes.c_double(0.0)
    _check(_lib.mertens_get_param(key.encode(), ctypes.byref(v)), f"mertens_get_param({key})")
    return v.value


def tuning() -> dict:
    """The tuning parameters the library currently runs with."""
    return {k: get_param(k) for k in TUNING_KEYS}


def set_stream(stream_handle: int | None) -> None:
    """Run on a HIP stream given as an integer handle (e.g. torch's cuda_stream)."""
    _check(_lib.mertens_set_stream(ctypes.c_void_p(stream_handle or 0)), "mertens_set_stream")


def stats() -> dict:
    vals = (ctypes.c_double * len(STAT_NAMES))()
    k = _lib.mertens_stats(vals, len(STAT_NAMES))
    return {STAT_NAMES[i]: vals[i] for i in range(k)}


def debug_div(n, d, on_device: bool) -> np.ndarray:
    na = np.ascontiguousarray(np.asarray(n, dtype=np.uint64))
    da = np.ascontiguousarray(np.asarray(d, dtype=np.uint64))
    assert na.shape == da.shape
    q = np.zeros(na.size, dtype=np.uint64)
    _check(_lib.mertens_debug_div(_u64p(na), _u64p(da), na.size, _u64p(q), int(on_device)),
           "mertens_debug_div")
    return q


def debug_wide(ms, ds, op: int, on_device: bool) -> list:
    """The wide-entry quotient routines on Python ints m (< 2^128) and d (< 2^64)."""
    lo = np.array([int(m) & (2**64 - 1) for m in ms], dtype=np.uint64)
    hi = np.array([int(m) >> 64 for m in ms], dtype=np.uint64)
    d = np.array([int(v) for v in ds], dtype=np.uint64)
    qlo = np.zeros(len(lo), dtype=np.uint64)
    qhi = np.zeros(len(lo), dtype=np.uint64)
    _check(_lib.mertens_debug_wide(_u64p(lo), _u64p(hi), _u64p(d), len(lo), _u64p(qlo), _u64p(qhi),
                                   op, int(on_device)), "mertens_debug_wide")
    return [(int(h) << 64) | int(l) for l, h in zip(qlo, qhi)]


def debug_runsum(n: int, L: int) -> int:
    """sum_{k > L} M(floor(n/k)) mod 2^64 by the plain grouped sweep."""
    out = _u64(0)
    _check(_lib.mertens_debug_runsum(n & (2**64 - 1), n >> 64, L, ctypes.byref(out)),
           "mertens_debug_runsum")
    return int(out.value)


def debug_primes(limit: int):
    """(count, largest, sum) of the primes 5 <= p <= limit of the host table."""
    c, l, t = _u64(0), _u64(0), _u64(0)
    _check(_lib.mertens_debug_primes(limit, ctypes.byref(c), ctypes.byref(l), ctypes.byref(t)),
           "mertens_debug_primes")
    return int(c.value), int(l.value), int(t.value)


def debug_mu(y1: int, count: int, with_sums: bool = True):
    mu = np.zeros(count, dtype=np.int8)
    sums = np.zeros(count, dtype=np.int64) if with_sums else None
    _check(_lib.mertens_debug_mu(y1, count, mu.ctypes.data_as(_P(ctypes.c_int8)),
                                 _i64p(sums) if with_sums else None), "mertens_debug_mu")
    return mu, sums


def raw():
    """The ctypes library handle (tests use it to probe error returns)."""
    return _lib
