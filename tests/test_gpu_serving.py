"""GPU tests of the serving path (mertens_submit / mertens_poll).

Requests share one running sieve sweep and join it at block boundaries;
every result must equal the oracle's (golden values) and mertens_query's,
alone or in the mix.
"""
from __future__ import annotations

import json
import os
import time

import pytest

from paper_1108_0135_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "golden.json")))


@pytest.fixture()
def mt():
    from paper_1108_0135_amd import mertens as mt
    mt.init(0, 1 << 24)  # small blocks: many block boundaries to join at
    yield mt
    mt.shutdown()


def _collect(mt, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = mt.poll(t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "serving did not finish"
        time.sleep(0.002)
    return out


def test_mix_matches_alone_and_oracle(mt):
    ns = GOLDEN["batch48"]["n"] + GOLDEN["seeded32"]["n"][:8] + [10**12]
    exp = GOLDEN["batch48"]["M"] + GOLDEN["seeded32"]["M"][:8] + [GOLDEN["n1e12"]["M"]]
    tickets = [mt.submit(n) for n in ns]
    assert all(t is not None for t in tickets)
    got = _collect(mt, tickets)
    assert [got[t][0] for t in tickets] == exp
    assert all(got[t][1] >= 0 for t in tickets)
    # the same values one request at a time, and through the synchronous path
    for n, e in zip(ns[::9], exp[::9]):
        t = mt.submit(n)
        assert _collect(mt, [t])[t][0] == e
        assert int(mt.query([n])[0]) == e


def test_staggered_arrivals_join_running_sweep(mt):
    g = GOLDEN["n1e16_samples"]
    big = [10**16 // c for c in g["c"][:4]]  # ~5e10..1e12: several blocks each
    first = [mt.submit(n) for n in big[:2]]
    time.sleep(0.05)
    second = [mt.submit(n) for n in big[2:]] + [mt.submit(n) for n in GOLDEN["batch48"]["n"][:6]]
    got = _collect(mt, first + second)
    assert [got[t][0] for t in first + second] == g["M"][:4] + GOLDEN["batch48"]["M"][:6]


def test_capacity_and_zero(mt):
    mt.set_param("serve_capacity", 2)
    a = mt.submit(GOLDEN["n1e12"]["n"])
    b = mt.submit(GOLDEN["n1e12"]["n"])
    assert a is not None and b is not None
    assert mt.submit(12345) is None  # no free slot: EAGAIN
    got = _collect(mt, [a, b])
    assert got[a][0] == got[b][0] == GOLDEN["n1e12"]["M"]
    z = mt.submit(0)
    assert _collect(mt, [z])[z] == (0, 0.0)
    with pytest.raises(Exception):
        mt.poll(z)  # already collected


def test_short_request_overtakes_long_sweep(mt):
    # a long request keeps the main sweep busy for thousands of 2^24-y blocks;
    # a short one rides the short sweep and finishes first, with its exact value
    long_t = mt.submit(10**17)
    time.sleep(0.1)
    short_n = GOLDEN["seeded32"]["n"][0]
    short_t = mt.submit(short_n)
    got = _collect(mt, [short_t])
    assert got[short_t][0] == GOLDEN["seeded32"]["M"][0]
    assert mt.poll(long_t) is None  # still sweeping
    assert _collect(mt, [long_t], timeout=300)[long_t][0] == inputs.TABLE1[10**17]


def test_bad_request_beside_good_ones(mt):
    # with an explicit small u, an n whose array would need 2^31 or more
    # entries is refused at submission; the requests around it complete
    # exactly and the worker keeps serving
    from paper_1108_0135_amd import mertens as binding
    mt.init(1000, 1 << 20)
    good = GOLDEN["seeded32"]["n"][:6]
    tickets = [mt.submit(n) for n in good[:3]]
    with pytest.raises(binding.MertensError) as err:
        mt.submit(10**13)  # L = 10^10 >= 2^31
    assert err.value.code == binding.EINVAL
    tickets += [mt.submit(n) for n in good[3:]]
    got = _collect(mt, tickets)
    assert [got[t][0] for t in tickets] == GOLDEN["seeded32"]["M"][:6]
    t = mt.submit(GOLDEN["batch48"]["n"][0])
    assert _collect(mt, [t])[t][0] == GOLDEN["batch48"]["M"][0]
