"""Autotuner of the library's performance parameters (results never depend on them).

Coordinate search through the C ABI on two calibration workloads:

* stage 1, the single query M(10^16) with u = 5*10^10 and y-blocks of 2^30:
  ``beta`` (split of each x's sum between the run-length part and the
  explicit k part), the work-item sizes ``ychunk`` / ``kchunk``, the
  persistent update grid ``waves_per_cu``, the band ``band_lo`` /
  ``band_hi`` of explicit-k reads summed y-major from LDS windows, how many
  blocks the sieve may run ahead of the update (``sieve_ahead``), and
  ``graph`` (one captured hipGraph of the block pipeline replayed per
  block, or direct launches);
* stage 2, the batched workload (256 n log-uniform in [1e13, 1e17], seed 0,
  plus 1e16 and 1e17) with automatic u and block: ``u_scale`` (automatic
  u = u_scale * (sum of n)^(2/3): the sieve costs ~u, the update
  ~(sum of n)/sqrt(u)), ``block_auto`` (the block length used when
  mertens_init gets block = 0), ``bucket_min`` (how many sieving primes
  above 2^17 a block needs before their multiples go through per-segment
  buckets) and ``graph`` again.

Every setting must give the same result bits (the tuner asserts it).  The
choice is written next to the library as ``tuned_<arch>.json`` together with
the SHA-256 of the kernel sources it was measured on; mertens_init applies
it when that hash equals the one compiled into the library, and ignores it
otherwise.

Usage: python -m paper_1108_0135_amd.autotune
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

from . import inputs
from . import mertens as mt

ARCH = os.environ.get("MERTENS_OFFLOAD_ARCH", "gfx950")
PKG = os.path.dirname(os.path.abspath(__file__))
TUNED_PATH = os.path.join(PKG, f"tuned_{ARCH}.json")
KERNEL_SOURCES = ("mertens_kernels.hip", "mertens_internal.h")

STAGE1 = {
    "beta": [0.15, 0.2, 0.25, 0.3, 0.4],
    "ychunk": [8192, 16384, 32768],
    "kchunk": [512, 1024, 2048],
    "waves_per_cu": [8, 12, 16],
    "band_lo": [0, 19, 21],
    "band_hi": [26, 27, 29],
    "sieve_ahead": [4, 16, 64],
    "graph": [0, 1],
}
STAGE2 = {
    "u_scale": [0.3, 0.4, 0.5, 0.65, 0.8, 1.0],
    "block_auto": [2**28, 2**29, 2**30, 2**31],
    "bucket_min": [2**14, 2**16, 2**18, 2**20],
    "graph": [0, 1],
}
KEYS = sorted(set(STAGE1) | set(STAGE2))
MIN_GAIN = 0.005  # relative gain a trial needs to replace the best setting


def kernel_source_sha256() -> str:
    """SHA-256 over the kernel sources (the build compiles the same value in)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _run(workload: str, params: dict, reps: int):
    """Best wall time of `reps` timed runs of the workload under params, and its results."""
    if workload == "n1e16":
        mt.init(5 * 10**10, 1 << 30)
        ns = [10**16]
    else:
        mt.init(0, 0)
        ns = [int(v) for v in inputs.batch_log_uniform(seed=0, count=256, lo=1e13, hi=1e17)]
        ns += [10**16, 10**17]
    try:
        for k, v in params.items():
            mt.set_param(k, v)
        ref = mt.query(ns if workload == "n1e16" else ns[:2])  # allocations, prime table
        best, res = float("inf"), None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = mt.query(ns)
            best = min(best, time.perf_counter() - t0)
        if workload == "n1e16" and int(res[0]) != inputs.TABLE1[10**16]:
            raise AssertionError("M(1e16) wrong under " + json.dumps(params))
        del ref
        return best, [int(v) for v in res]
    finally:
        mt.shutdown()


def _stage(workload: str, space: dict, params: dict, reps: int, log) -> tuple[dict, float]:
    t_best, ref = _run(workload, params, reps)
    log(f"{workload}: start {json.dumps(params)} {t_best * 1e3:.1f} ms")
    for key, values in space.items():
        for v in values:
            if v == params.get(key):
                continue
            trial = dict(params, **{key: v})
            t, res = _run(workload, trial, reps)
            if res != ref:
                raise AssertionError(f"{key}={v} changed a result")
            log(f"{workload}: {key}={v}: {t * 1e3:.1f} ms (best {t_best * 1e3:.1f})")
            # a setting moves only on a gain above run-to-run noise (so that,
            # e.g., a deeper sieve ring that buys nothing holds no memory)
            if t < t_best * (1.0 - MIN_GAIN):
                t_best, params = t, trial
    return params, t_best


def defaults() -> dict:
    """The library's built-in values of the tuned keys (no tuned file applied)."""
    mt.init(0, 0)
    try:
        return {k: mt.get_param(k) for k in KEYS}
    finally:
        mt.shutdown()


def calibrate(verbose: bool = True) -> dict:
    log = (lambda s: print(s, flush=True)) if verbose else (lambda s: None)
    os.environ["MERTENS_TUNED"] = "0"  # measure from the built-in defaults
    params = defaults()
    params, t1 = _stage("n1e16", STAGE1, params, reps=3, log=log)
    params, t2 = _stage("batched", STAGE2, params, reps=1, log=log)
    out = {"arch": ARCH, "source_sha256": kernel_source_sha256(), "params": params,
           "seconds": {"n1e16": t1, "batched": t2},
           "workloads": {"n1e16": "M(1e16), u = 5e10, y-blocks of 2^30",
                         "batched": "256 n log-uniform in [1e13, 1e17] (seed 0) + 1e16 + 1e17, "
                                    "automatic u and block"}}
    with open(TUNED_PATH, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load(path: str = TUNED_PATH) -> dict:
    """The stored parameters (empty when absent or taken on other kernel sources)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    return d["params"] if d.get("source_sha256") == kernel_source_sha256() else {}


if __name__ == "__main__":
    print(json.dumps(calibrate()))
