"""Plain CPU oracle for the Mertens function (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its binding) never imports, links or calls it, and the two share
no code: the oracle is compiled from ``mertens_oracle.c`` with gcc.

Tiers (see the C file for the paper passages each follows):

* O1 ``mu_range``, ``mertens_table``, ``mertens_many`` -- the exact block
  sieve of Section 3 (products of -p, zero on p^2, sign test), summed in
  order (Section 1 definition of M).
* O2 ``mertens_identity`` -- the Section 2 identity with a threshold t,
  evaluated recursively on top of an O1 table M(0..T).
* O3 ``interval`` -- Section 6: M over [a, b] from an exact M(a) and the O1
  sieve, with the extremes of M(n)/sqrt(n) compared exactly.

Parity pins for every tier live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mertens_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_default = None


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (plain C, -O2, single-threaded)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


class OracleLib:
    """ctypes view of one compiled oracle (the default one, or a test build)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        u64, i64p = ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)
        lib.oracle_mu_range.argtypes = [u64, u64, ctypes.POINTER(ctypes.c_int8)]
        lib.oracle_mertens_table.argtypes = [u64, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_mertens_many.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t, i64p]
        lib.oracle_mertens_identity.argtypes = [u64, ctypes.POINTER(ctypes.c_int32), u64, i64p, i64p, u64]
        lib.oracle_interval.argtypes = [u64, u64, ctypes.c_int64, i64p,
                                        ctypes.POINTER(ctypes.c_uint64), i64p]
        lib.oracle_isqrt.argtypes = [u64]
        lib.oracle_isqrt.restype = u64
        for f in ("oracle_mu_range", "oracle_mertens_table", "oracle_mertens_many",
                  "oracle_mertens_identity", "oracle_interval"):
            getattr(lib, f).restype = ctypes.c_int
        self.lib = lib

    def mu_range(self, y1: int, y2: int) -> np.ndarray:
        """mu(y) for y in [y1, y2] as int8 (mu(0) = 0 by convention)."""
        out = np.empty(y2 - y1 + 1, dtype=np.int8)
        _check(self.lib.oracle_mu_range(y1, y2, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))),
               "mu_range")
        return out

    def mertens_table(self, N: int) -> np.ndarray:
        """M(0..N) as int32 (M(0) = 0)."""
        tab = np.empty(N + 1, dtype=np.int32)
        _check(self.lib.oracle_mertens_table(N, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "mertens_table")
        return tab

    def mertens_many(self, ns) -> np.ndarray:
        """M(n) for every n in ``ns`` by one O1 sieve sweep to max(ns)."""
        arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
        out = np.empty(arr.size, dtype=np.int64)
        if arr.size:
            _check(self.lib.oracle_mertens_many(
                arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), arr.size,
                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "mertens_many")
        return out

    def identity(self, n: int, tab: np.ndarray, L: int = 0):
        """O2: (M(n), [M(floor(n/c)) for c = 1..L]) from the table tab = M(0..T)."""
        mn = ctypes.c_int64(0)
        byp = np.empty(max(L, 1), dtype=np.int64)
        _check(self.lib.oracle_mertens_identity(
            n, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), tab.size - 1,
            ctypes.byref(mn), byp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), L),
            "mertens_identity")
        return int(mn.value), byp[:L].copy()


    def interval(self, a: int, b: int, m_a: int) -> dict:
        """O3: from M(a), M(b) and the extremes of M(n)/sqrt(n) over n in [a, b]."""
        m_b = ctypes.c_int64(0)
        n_ext = (ctypes.c_uint64 * 2)()
        m_ext = (ctypes.c_int64 * 2)()
        _check(self.lib.oracle_interval(a, b, m_a, ctypes.byref(m_b), n_ext, m_ext), "interval")
        return {"m_b": int(m_b.value), "n_min": int(n_ext[0]), "m_min": int(m_ext[0]),
                "n_max": int(n_ext[1]), "m_max": int(m_ext[1])}


def default() -> OracleLib:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build()
        _default = OracleLib(_LIB)
    return _default


def mu_range(y1: int, y2: int) -> np.ndarray:
    return default().mu_range(y1, y2)


def mertens_table(N: int) -> np.ndarray:
    return default().mertens_table(N)


def mertens_many(ns) -> np.ndarray:
    return default().mertens_many(ns)


def interval(a: int, b: int, m_a: int) -> dict:
    return default().interval(a, b, m_a)


def isqrt(v: int) -> int:
    return int(default().lib.oracle_isqrt(v))


def table_size_for(n: int) -> int:
    """A table bound T for O2: about n^(2/3), never below floor(sqrt(n))."""
    return max(isqrt(n), int(round(n ** (2.0 / 3.0))), 16)


class IdentityOracle:
    """O2 with one shared O1 table M(0..T); answers many n <= T^2."""

    def __init__(self, T: int, lib: OracleLib | None = None):
        self.T = int(T)
        self.lib = lib or default()
        self.tab = self.lib.mertens_table(self.T)

    def query(self, n: int, L: int = 0):
        """Return (M(n), byproducts) where byproducts[c-1] = M(floor(n/c)), c = 1..L."""
        return self.lib.identity(n, self.tab, L)


def mertens(n: int) -> int:
    """M(n) by the cheapest oracle tier that reaches n."""
    if n <= 2_000_000:
        return int(mertens_many([n])[0])
    return IdentityOracle(table_size_for(n)).query(n)[0]
