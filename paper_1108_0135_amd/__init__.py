"""MI355X-native exact Mertens function M(n) (arXiv:1108.0135 method).

The compute path is the HIP library ``libmertens.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/mertens.h``; ``paper_1108_0135_amd.mertens``
is its thin ctypes binding.  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
