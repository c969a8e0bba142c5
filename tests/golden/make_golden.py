"""Write the stored expected values used by the GPU parity tests.

Calls only the CPU oracle (``oracle/``) on the seeded inputs of
``paper_1108_0135_amd.inputs``; never the GPU path.  Re-run after any change
to the oracle's arithmetic:  python tests/golden/make_golden.py
(``--only-intervals tests/golden/golden.json`` refreshes just the interval
entries of an existing file, ``--only-batch256 tests/golden/golden.json``
just the batched-workload entries.)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1108_0135_amd import inputs  # noqa: E402


def interval_cases(out: dict) -> None:
    """Section 6 interval sweeps (O3 on top of O2 or of the paper's value)."""
    # a ragged interval of 3 * 2^20 + 12346 values at a height of ~1e12 (seed 3)
    a, b = inputs.interval_around(3, 10**12, 2 * 10**12, 0, 3 * 2**20 + 12345)
    o2 = oracle.IdentityOracle(10**8)
    m_a = o2.query(a)[0]
    r = oracle.interval(a, b, m_a)
    assert r["m_b"] == o2.query(b)[0]  # the two tiers agree at the far end
    out["interval1e12"] = {"seed": 3, "a": a, "b": b, "m_a": m_a, **r}

    # the neighbourhood of the Section 6 extreme: M(a) from the printed
    # M(EXTREME_N) minus the oracle's mu over (a, EXTREME_N], then O3
    a, b = inputs.extreme_window()
    mu = oracle.mu_range(a, b).astype(np.int64)  # mu[i] = mu(a + i)
    m_a = inputs.EXTREME_M - int(mu[1:inputs.EXTREME_N - a + 1].sum())
    r = oracle.interval(a, b, m_a)
    assert (r["n_min"], r["m_min"]) == (inputs.EXTREME_N, inputs.EXTREME_M)
    rng = np.random.default_rng(8)
    idx = sorted(int(i) for i in rng.choice(b - a + 1, 64, replace=False))
    run = m_a + np.cumsum(mu[1:])  # run[i - 1] = M(a + i)
    samples = {str(a + i): (m_a if i == 0 else int(run[i - 1])) for i in idx}
    out["extreme_window"] = {"a": a, "b": b, "m_a": m_a, **r, "samples": samples}


BATCH256_MAX = 3 * 10**14  # the members of the batched workload O2 reaches in minutes
BATCH256_BYP_C = 200        # byproducts c <= this of the largest such member


def _o2_worker(n: int) -> int:
    return _O2_SHARED.query(n)[0]


_O2_SHARED = None


def batch256_cases(out: dict, workers: int = 7, T: int = 4 * 10**9) -> None:
    """The batched workload (256 n log-uniform in [1e13, 1e17], seed 0): O2 for
    every member up to BATCH256_MAX, and sampled byproducts of the largest.

    One O1 table M(0..T) is built once and shared by forked worker processes
    (copy-on-write, read only); each O2 evaluation runs single-threaded."""
    import multiprocessing as mp
    global _O2_SHARED
    ns = [int(v) for v in inputs.batch_log_uniform(seed=0, count=256, lo=1e13, hi=1e17)]
    idx = [i for i, n in enumerate(ns) if n <= BATCH256_MAX]
    _O2_SHARED = oracle.IdentityOracle(T)
    order = sorted(idx, key=lambda i: -ns[i])  # largest first: better balance
    with mp.get_context("fork").Pool(workers) as pool:
        vals = pool.map(_o2_worker, [ns[i] for i in order], chunksize=1)
    got = dict(zip(order, vals))
    big = max(idx, key=lambda i: ns[i])
    rng = np.random.default_rng(11)
    cs = sorted({int(c) for c in rng.integers(2, BATCH256_BYP_C + 1, 12)} | {2, BATCH256_BYP_C})
    m, byp = _O2_SHARED.query(ns[big], BATCH256_BYP_C)
    assert m == got[big]
    out["batch256"] = {"seed": 0, "max_n": BATCH256_MAX, "index": idx,
                       "n": [ns[i] for i in idx], "M": [int(got[i]) for i in idx],
                       "byproducts_of": big, "c": cs, "byproducts": [int(byp[c - 1]) for c in cs]}
    _O2_SHARED = None


def main() -> None:
    t0 = time.time()
    if len(sys.argv) > 2 and sys.argv[1] == "--only-intervals":
        # refresh only the interval entries of an existing file
        path = sys.argv[2]
        out = json.load(open(path))
        interval_cases(out)
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"updated {path} in {time.time() - t0:.1f} s")
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--only-batch256":
        path = sys.argv[2]
        out = json.load(open(path))
        batch256_cases(out)
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"updated {path} in {time.time() - t0:.1f} s")
        return
    out = {"generator": "tests/golden/make_golden.py (oracle only)"}

    # the brute-force-checkable set: 32 n uniform in [2, 1e9], seed 0 (O1 sweep)
    ns = inputs.uniform_small(seed=0, count=32)
    out["seeded32"] = {"seed": 0, "n": [int(v) for v in ns],
                       "M": [int(v) for v in oracle.mertens_many(ns)]}

    # n = 1e12 and every byproduct M(floor(n/c)), c <= 1e4 (O2 on an O1 table to 1e8)
    o2 = oracle.IdentityOracle(10**8)
    m, byp = o2.query(10**12, 10**4)
    out["n1e12"] = {"n": 10**12, "L": 10**4, "M": m, "byproducts": [int(v) for v in byp]}

    # n = 1e16, u = 5e10 (L = 2e5): sampled byproducts c in [1e4, 2e5] that O2 reaches
    rng = np.random.default_rng(5)
    cs = sorted({int(c) for c in rng.integers(10**4, 2 * 10**5 + 1, 12)} | {10**4, 2 * 10**5})
    out["n1e16_samples"] = {"n": 10**16, "c": cs,
                            "M": [o2.query(10**16 // c)[0] for c in cs]}

    # a mixed batch: 48 n log-uniform in [1e3, 1e11], seed 1
    nb = inputs.log_uniform(1, 48, 1e3, 1e11)
    out["batch48"] = {"seed": 1, "n": [int(v) for v in nb],
                      "M": [o2.query(int(v))[0] for v in nb]}

    # a dense window: n_i = n0 + 997 i, i < 8, n0 uniform in [1e12, 2e12] (seed 2)
    nw = inputs.dense_window(seed=2, count=8, lo=10**12, hi=2 * 10**12)
    out["window1e12"] = {"seed": 2, "n": [int(v) for v in nw],
                         "M": [o2.query(int(v))[0] for v in nw]}

    # the dense window at full size (n0 from seed 0 in [1e18, 1.8e19]): the
    # differences M(n_{i+1}) - M(n_i) = sum of mu over (n_i, n_{i+1}], i < 7
    # (O1 on the window; the M(n_i) themselves are beyond the oracle)
    nd = [int(v) for v in inputs.dense_window(seed=0, count=8)]
    mu = oracle.mu_range(nd[0] + 1, nd[-1])
    diffs = [int(mu[nd[i] - nd[0]:nd[i + 1] - nd[0]].astype(np.int64).sum()) for i in range(7)]
    out["window1e19_diffs"] = {"seed": 0, "n": nd, "diffs": diffs}

    interval_cases(out)
    batch256_cases(out)

    path = os.path.join(HERE, "golden.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
