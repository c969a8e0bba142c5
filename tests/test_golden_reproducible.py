"""The stored expected values are the oracle's: recompute the cheap ones.

tests/golden/golden.json is written by tests/golden/make_golden.py from the
oracle alone.  These CPU tests recompute the entries that take seconds (the
inputs from their seeds, then the oracle) and require the stored values.
"""
from __future__ import annotations

import json
import os

import pytest

import oracle
from paper_1108_0135_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "golden.json")))


@pytest.fixture(scope="module")
def o2():
    return oracle.IdentityOracle(10**8)


def test_seeded32_inputs_and_values():
    g = GOLDEN["seeded32"]
    ns = [int(v) for v in inputs.uniform_small(seed=g["seed"], count=32)]
    assert ns == g["n"]
    assert [int(v) for v in oracle.mertens_many(ns)] == g["M"]


def test_n1e12_and_window1e12(o2):
    g = GOLDEN["n1e12"]
    m, byp = o2.query(g["n"], g["L"])
    assert m == g["M"] and [int(v) for v in byp] == g["byproducts"]
    w = GOLDEN["window1e12"]
    ns = [int(v) for v in inputs.dense_window(seed=w["seed"], count=8, lo=10**12, hi=2 * 10**12)]
    assert ns == w["n"]
    assert [o2.query(n)[0] for n in ns] == w["M"]


def test_interval1e12(o2):
    g = GOLDEN["interval1e12"]
    a, b = inputs.interval_around(g["seed"], 10**12, 2 * 10**12, 0, 3 * 2**20 + 12345)
    assert (a, b) == (g["a"], g["b"])
    m_a = o2.query(a)[0]
    assert m_a == g["m_a"]
    r = oracle.interval(a, b, m_a)
    assert r == {k: g[k] for k in ("m_b", "n_min", "m_min", "n_max", "m_max")}
    assert o2.query(b)[0] == g["m_b"]


def test_batch256_smallest_member():
    # the batched workload's goldens: the inputs from their seed, and the
    # smallest member's M(n) recomputed by O2 (about 15 s)
    g = GOLDEN["batch256"]
    ns = [int(v) for v in inputs.batch_log_uniform(seed=g["seed"], count=256, lo=1e13, hi=1e17)]
    assert [ns[i] for i in g["index"]] == g["n"]
    assert g["index"] == [i for i, n in enumerate(ns) if n <= g["max_n"]]
    k = min(range(len(g["n"])), key=lambda i: g["n"][i])
    assert oracle.IdentityOracle(3 * 10**8).query(g["n"][k])[0] == g["M"][k]
