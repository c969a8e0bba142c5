"""GPU test of mertens_query_noalloc, the entry point that allocates no device
memory (its buffers are pieces of one static device array): the same values
as mertens_query on two calls in a row, the second smaller, and a clear
error for a request beyond the scratch."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from paper_1108_0135_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "golden.json")))


def test_noalloc_matches_query_twice_then_smaller():
    from paper_1108_0135_amd import mertens as mt
    mt.init(0, 0)
    try:
        big = GOLDEN["batch48"]["n"] + [10**12, 10**13 + 7, 0]
        small = GOLDEN["seeded32"]["n"][:5]
        want_big = mt.query(big)
        got_big = mt.query_noalloc(big)
        assert np.array_equal(got_big, want_big)
        assert list(got_big[:48]) == GOLDEN["batch48"]["M"]
        assert int(got_big[48]) == GOLDEN["n1e12"]["M"]
        # byproducts still refer to the last allocating query (its 10^12)
        L = mt.byproducts(48).size
        assert list(mt.byproducts(48, min(L, 100))) == GOLDEN["n1e12"]["byproducts"][:min(L, 100)]
        want_small = mt.query(small)
        got_small = mt.query_noalloc(small)
        assert np.array_equal(got_small, want_small)
        assert list(got_small) == GOLDEN["seeded32"]["M"][:5]
        # a request beyond the scratch: a clear error, the next call still works
        with pytest.raises(mt.MertensError) as err:
            mt.query_noalloc([10**19])
        assert err.value.code == mt.ENOMEM and "scratch" in str(err.value)
        assert np.array_equal(mt.query_noalloc(small), want_small)
        assert int(mt.query_noalloc([10**16])[0]) == inputs.TABLE1[10**16]
    finally:
        mt.shutdown()
