"""Benchmark: exact M(n) on one MI355X through the HIP C ABI.

A step is one full pass of the hot path for the workload n = 10^16 with
u = 5*10^10 and y-blocks of 2^30 (47 blocks, L = 2*10^5 byproducts):
block sieve -> M(y) prefix scan -> per-block contribution update ->
finalize.  The metric is sieved y per second through the update (the
sweep covers y in [0, floor(n/(L+1))]); the step's result is checked
against Table 1 of the paper before timing.

Prints ONE JSON line (see the repository's benchmark contract).  The
`roofline` object is for the dominant kernel, timed with HIP events on the
library's own stream; `cpu_baseline` times the CPU oracle on a bounded
sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_WORK = 10**16
U_WORK = 5 * 10**10
BLOCK_WORK = 1 << 30
EXPECTED = -3195437  # Table 1 of the paper

# MI355X published peaks used for the roofline
HBM_PEAK_GBS = 8000.0
CU, CLOCK_GHZ, LANES = 256, 2.4, 64
INT_VALU_PEAK_TOPS = CU * LANES * CLOCK_GHZ / 1000.0  # 39.3 T int32 lane-ops/s
# algorithmic cost of one quotient floor(m/d) by an invariant divisor plus its
# accumulation, in full-rate int32 lane-op equivalents: 4 32x32->64 products
# (quarter rate, 4 slots each) + 8 add/sub/shift ops
OPS_PER_QUOTIENT = 24


def cpu_baseline(budget_s: float = 15.0) -> dict:
    """The oracle's exact block sieve (O1) over [1, N] on one host core."""
    import oracle
    oracle.build()
    lib = oracle.default()
    N = 2 * 10**8
    t0 = time.perf_counter()
    lib.mertens_many([N])
    dt = time.perf_counter() - t0
    reps = 1
    while dt * (reps + 1) / reps < budget_s and reps < 8:
        t1 = time.perf_counter()
        lib.mertens_many([N])
        dt += time.perf_counter() - t1
        reps += 1
    return {"value": N * reps / dt, "unit": "sieved y/s", "cores": 1, "kind": "oracle",
            "sample": f"O1 exact block sieve + running sum of y in [1, {N:.0e}] x{reps} "
                      f"(single thread, {dt:.1f} s); the oracle has no update step, and its "
                      f"M(1e16) would need the whole [1, 1e16] sieved"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the sweep would shard)", file=sys.stderr)
        return 2

    import torch
    from paper_1108_0135_amd import mertens as mt

    mt.init(U_WORK, BLOCK_WORK)
    for _ in range(max(args.warmup, 1)):
        got = int(mt.query([N_WORK])[0])
        if got != EXPECTED:
            print(f"wrong result M(1e16) = {got}, expected {EXPECTED}", file=sys.stderr)
            return 1

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kstats = []
    for _ in range(args.steps):
        r = int(mt.query([N_WORK])[0])
        kstats.append(mt.stats())
        if r != EXPECTED:
            print(f"wrong result in timed step: {r}", file=sys.stderr)
            return 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1000.0 * dt / args.steps
    st = kstats[-1]
    sieved = st["sieved_y"]

    def avg(key):
        return sum(s[key] for s in kstats) / len(kstats)

    launches = st["update_launches"]
    upd_ms_launch = avg("ms_update") / launches
    sieve_ms_launch = avg("ms_sieve") / st["sieve_launches"]
    quot = st["rl_quotients"] + st["k_quotients"]
    upd_tops = quot / launches * OPS_PER_QUOTIENT / (upd_ms_launch * 1e-3) / 1e12
    # sieve kernel: HBM bytes it must write per y (two 64-bit masks per 64 y)
    sieve_gbs = (sieved / st["sieve_launches"]) * 0.25 / (sieve_ms_launch * 1e-3) / 1e9
    if avg("ms_update") >= avg("ms_sieve"):
        roof = {"kernel": "k_update", "bound": "alu", "achieved": upd_tops,
                "peak": INT_VALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": upd_tops / INT_VALU_PEAK_TOPS, "traffic": None,
                "avg_launch_ms": upd_ms_launch, "launches": launches,
                "quotients_per_launch": quot / launches}
    else:
        roof = {"kernel": "k_sieve", "bound": "hbm", "achieved": sieve_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sieve_gbs / HBM_PEAK_GBS,
                "traffic": None, "avg_launch_ms": sieve_ms_launch,
                "launches": st["sieve_launches"]}

    line = {
        "metric": "sieved y/sec through update; batched vs plain M(n) queries/sec, 1 GPU, exact",
        "value": sieved / (ms_step * 1e-3),
        "unit": "sieved y/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain single query n=1e16, u=5e10, y-blocks of 2^30 "
                               "(47 blocks, L=2e5, all byproducts)",
                   "n": N_WORK, "u": U_WORK, "block": BLOCK_WORK, "sieved_y": sieved,
                   "parallelism": "1 GPU"},
        "plain_queries_per_s": 1000.0 / ms_step,
        "kernel_ms": {k: avg(k) for k in ("ms_sieve", "ms_scan", "ms_prep", "ms_update",
                                          "ms_finalize", "ms_total")},
        "quotients": {"run_length": st["rl_quotients"], "explicit_k": st["k_quotients"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    mt.shutdown()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
