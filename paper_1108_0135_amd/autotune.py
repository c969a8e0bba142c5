"""Autotuner for the update split and the sieve limit.

Times calibration queries through the C ABI and keeps, per parameter in
turn (coordinate search), the fastest value:

* ``beta``    -- split of each x's sum between the run-length part and the
  explicit k part (cheap fp64/integer quotients vs. M(y) gathers);
* ``u_scale`` -- the automatic u = u_scale * (sum of n)^(2/3): the sieve
  costs ~u, the update ~(sum of n)/sqrt(u), so only the ratio of the two
  measured rates matters and one scale serves every batch;
* ``ychunk`` / ``kchunk`` -- work-item sizes of the persistent update.

Every setting must give the same result bits (the parameters are pure
performance knobs); the tuner asserts it.  The choice is stored as JSON
next to the library (``tuned_<arch>.json``) and applied by ``apply()``.

Usage: python -m paper_1108_0135_amd.autotune [n]
"""
from __future__ import annotations

import json
import os
import sys
import time

from . import mertens as mt

ARCH = os.environ.get("MERTENS_OFFLOAD_ARCH", "gfx950")
TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"tuned_{ARCH}.json")

DEFAULTS = {"beta": 0.25, "u_scale": 0.5, "ychunk": 16384, "kchunk": 1024}
SPACE = {
    "beta": [0.15, 0.2, 0.25, 0.3, 0.4],
    "u_scale": [0.3, 0.4, 0.5, 0.65, 0.8, 1.0],
    "ychunk": [4096, 8192, 16384, 32768],
    "kchunk": [512, 1024, 2048],
}


def _time_query(ns, params, reps=2):
    mt.init(0, 0)
    for k, v in params.items():
        mt.set_param(k, v)
    res = mt.query(ns)  # warm (allocations, prime table)
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        r = mt.query(ns)
        best = min(best, time.perf_counter() - t0)
        assert (r == res).all(), "tuning changed a result"
    mt.shutdown()
    return best, [int(v) for v in res]


def calibrate(ns=(10**15,), reps=2, verbose=True) -> dict:
    ns = [int(v) for v in ns]
    params = dict(DEFAULTS)
    t_best, ref = _time_query(ns, params, reps)
    trail = [{"params": dict(params), "s": t_best}]
    for key, values in SPACE.items():
        for v in values:
            if v == params[key]:
                continue
            trial = dict(params, **{key: v})
            t, res = _time_query(ns, trial, reps)
            if res != ref:
                raise AssertionError(f"{key}={v} changed a result")
            trail.append({"params": trial, "s": t})
            if verbose:
                print(f"  {key}={v}: {t * 1e3:.1f} ms (best {t_best * 1e3:.1f})", flush=True)
            if t < t_best:
                t_best, params = t, trial
    out = {"arch": ARCH, "calibration_n": ns, "params": params, "seconds": t_best,
           "trials": len(trail)}
    with open(TUNED_PATH, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load(path: str = TUNED_PATH) -> dict:
    if not os.path.exists(path):
        return dict(DEFAULTS)
    with open(path) as f:
        return json.load(f)["params"]


def apply(path: str = TUNED_PATH) -> dict:
    """Set the stored parameters on the current context (after mertens.init)."""
    params = load(path)
    for k, v in params.items():
        mt.set_param(k, v)
    return params


if __name__ == "__main__":
    n = int(float(sys.argv[1])) if len(sys.argv) > 1 else 10**15
    print(json.dumps(calibrate([n])))
