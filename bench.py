"""Benchmark: exact M(n) on one MI355X through the HIP C ABI.

Default workload (the one line the contract asks for): a step is one full
pass of the hot path for n = 10^16 with u = 5*10^10 and y-blocks of 2^30
(47 blocks, L = 2*10^5 byproducts): block sieve -> M(y) prefix scan ->
per-block contribution update -> finalize.  The metric is sieved y per
second through the update (the sweep covers y in [0, floor(n/(L+1))]);
every step's result is checked against Table 1 of the paper.  The line also
carries the batched workload (256 n log-uniform in [1e13, 1e17] plus 1e16
and 1e17) as one shared sweep against one query at a time, the roofline of
the dominant kernel (HIP events on the library stream) and the CPU oracle
timed on the host (one core, and one process per core).

Other workloads (``--workload``), reported separately:
  batched  256 n log-uniform in [1e13, 1e17] (seed 0) plus 1e16 and 1e17,
           one shared sweep vs. one query at a time
  serving  Poisson arrivals at each of ``--rates`` q/s (``--count`` queries,
           n log-uniform in [1e10, 1e18]) through mertens_submit/poll vs. a
           one-at-a-time FIFO server; p50/p99 latency and queries/s per rate
  interval Section 6 localization: M(n) for every n of a 2^35-wide interval
           from the printed extreme on, and the extremes of M(n)/sqrt(n)
  wide     M(10^20) past the 64-bit limit (about 100 s per step; one timed
           step and no warmup unless asked)
  window   the dense window: 1024 n_i = n0 + 997 i near 1.2e19 as one shared
           sweep (one timed step), against the first member alone
"""
from __future__ import annotations

import argparse
import hashlib
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
METRIC = "sieved y/sec through update; batched vs plain M(n) queries/sec, 1 GPU, exact"

# MI355X published figures used for the roofline
HBM_PEAK_GBS = 8000.0
CU, CLOCK_GHZ, LANES = 256, 2.4, 64
INT_VALU_PEAK_TOPS = CU * LANES * CLOCK_GHZ / 1000.0  # 39.3 T int32 lane-ops/s
# algorithmic cost of one pair of the update, in full-rate VALU lane-ops: the
# quotient floor(m/d) (one fused multiply-add with a reciprocal of d) and its
# signed accumulation (one multiply-add); fp64 fma is full rate on MI355X
OPS_PER_QUOTIENT = 2
RECORD_BYTES = 16  # one sieve record: M(y) checkpoint and mu bits of 32 y
# the method's own need per explicit-k pair: one int32 M(y) read at a random y
GATHER_BYTES = 4


def kernel_source_sha256() -> str:
    """Hash of the kernel sources; counter summaries older than it do not apply."""
    h = hashlib.sha256()
    for name in ("mertens_kernels.hip", "mertens_internal.h"):
        with open(os.path.join(ROOT, "paper_1108_0135_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_per_launch(kernel: str, workload: str = "n1e16"):
    """HBM bytes per launch from the committed counter summary, or None if the
    kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_sha256():
        return None
    return d["hbm_bytes_per_launch"]


def progress(msg: str) -> None:
    """A progress line on stderr (long runs stay visibly alive)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """Host core count (usable by this process) and CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": usable, "cpu_count": os.cpu_count(), "model": model}


def _o2_child(conn, T: int, n: int) -> None:
    import oracle
    o2 = oracle.IdentityOracle(T)
    t0 = time.perf_counter()
    m = o2.query(n)[0]
    conn.send((m, time.perf_counter() - t0))
    conn.close()


def cpu_baseline(sieved_y: float, gpu_m_sample: int | None = None) -> dict:
    """The oracle per query, on the host cores.

    O2 (the Section 2 identity, recursively, on an O1 table M(0..T)) is
    timed on one core for M(10^12) with T = 10^8: 10^12 = 10^16 / 10^4 is
    the byproduct M(floor(n/c)) of the workload at c = 10^4, so this is a
    bounded piece of the same query.  The time for M(10^16) itself is
    extrapolated (labelled) from O2's cost, T for the table plus n / sqrt(T)
    for the recursion, at the largest table that fits a host comfortably
    (T = 2^31, 8 GiB).  `value` is the workload's sieved y (the GPU sweep's
    work for one M(10^16)) over that extrapolated oracle time, so it reads in
    the metric's unit.  The all-cores figure runs one O2 process per core on
    the same 10^12 query (queries are independent).  The oracle's M(10^12)
    must equal the GPU's byproduct at c = 10^4 (gpu_m_sample)."""
    import multiprocessing as mp
    import oracle
    oracle.build()
    T_s, n_s, T_big = 10**8, 10**12, 2**31
    t0 = time.perf_counter()
    o2 = oracle.IdentityOracle(T_s)
    t_table = time.perf_counter() - t0
    t0 = time.perf_counter()
    m_s = o2.query(n_s)[0]
    t_query = time.perf_counter() - t0
    if gpu_m_sample is not None and m_s != gpu_m_sample:
        raise RuntimeError(f"oracle M(1e12) = {m_s} differs from the GPU byproduct {gpu_m_sample}")
    # extrapolation: table linear in T; recursion proportional to n / sqrt(T)
    t_ext = t_table * T_big / T_s + t_query * (N_WORK / n_s) * (T_s / T_big) ** 0.5
    cpu = host_cpu()
    procs = max(1, min(cpu["nproc"], 16))
    ctx = mp.get_context("spawn")
    pipes, kids = [], []
    t0 = time.perf_counter()
    for _ in range(procs):
        a, b = ctx.Pipe(duplex=False)
        pr = ctx.Process(target=_o2_child, args=(b, T_s, n_s))
        pr.start()
        pipes.append(a)
        kids.append(pr)
    res = [a.recv() for a in pipes]
    for pr in kids:
        pr.join()
    t_all = time.perf_counter() - t0
    if any(m != m_s for m, _ in res):
        raise RuntimeError("oracle processes disagree")
    return {"value": sieved_y / t_ext, "unit": "sieved y/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"O2 single thread for M(1e12) = M(1e16 // 1e4), the workload's byproduct "
                       f"at c = 1e4: table T = 1e8 in {t_table:.2f} s + recursion {t_query:.2f} s; "
                       f"M(1e16) EXTRAPOLATED to {t_ext:.0f} s at T = 2^31 (table linear in T, "
                       f"recursion in n / sqrt(T)); value = the GPU sweep's {sieved_y:.3g} y "
                       f"for one M(1e16) over that time"),
            "per_query_s": {"n=1e12 measured (T=1e8, incl. table)": t_table + t_query,
                            "n=1e16 extrapolated (T=2^31)": t_ext},
            "all_cores": {"processes": procs, "wall_s": t_all,
                          "queries_per_s": procs / t_all,
                          "sample": f"{procs} independent O2 processes, each M(1e12) with its "
                                    f"own T = 1e8 table"},
            "host": cpu}


def batched_vs_plain(mt, ns) -> dict:
    """queries/s of one shared sweep vs. the same queries one at a time."""
    mt.init(0, 0)
    mt.query(ns[:2])  # warm
    t0 = time.perf_counter()
    plain = []
    for i, n in enumerate(ns):
        plain.append(int(mt.query([n])[0]))
        if i % 64 == 63:
            progress(f"one at a time: {i + 1} of {len(ns)}")
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batched = [int(v) for v in mt.query(ns)]
    t_batch = time.perf_counter() - t0
    if batched != plain:
        raise RuntimeError("batched results differ from one-at-a-time results")
    st = mt.stats()
    return {"queries": len(ns), "plain_qps": len(ns) / t_plain, "batched_qps": len(ns) / t_batch,
            "speedup": t_plain / t_batch, "plain_s": t_plain, "batched_s": t_batch,
            "batched_u": st["u"], "batched_sieved_y": st["sieved_y"],
            "batched_blocks": st["blocks"], "results": batched}


def workload_default(args, mt) -> dict:
    import torch

    progress("default workload: M(1e16)")
    mt.init(U_WORK, BLOCK_WORK)
    ahead = 1 if args.in_turn else int(mt.get_param("sieve_ahead"))  # the tuned value
    mt.set_param("sieve_ahead", ahead)
    for _ in range(max(args.warmup, 1)):
        got = int(mt.query([N_WORK])[0])
        if got != EXPECTED:
            raise RuntimeError(f"wrong result M(1e16) = {got}, expected {EXPECTED}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kstats = []
    for _ in range(args.steps):
        r = int(mt.query([N_WORK])[0])
        kstats.append(mt.stats())
        if r != EXPECTED:
            raise RuntimeError(f"wrong result in timed step: {r}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1000.0 * dt / args.steps
    st = kstats[-1]
    sieved = st["sieved_y"]

    def avg(key):
        return sum(s[key] for s in kstats) / len(kstats)

    # Per-kernel launch times for the roofline: one more query with the sieve
    # strictly in turn (sieve_ahead = 1), so no kernel's HIP-event interval
    # includes time shared with the other stream.  Not part of `value`.
    mt.set_param("sieve_ahead", 1)
    if int(mt.query([N_WORK])[0]) != EXPECTED:
        raise RuntimeError("wrong result in the in-turn pass")
    seq = mt.stats()
    mt.set_param("sieve_ahead", ahead)
    launches = seq["update_launches"]
    # the update step of a block is the persistent k_update and, where the
    # band applies (block 0 here), the y-major k_ek_window after it
    band_ms = seq.get("ms_band", 0.0)
    band_q = seq.get("band_quotients", 0.0)
    upd_ms_total = seq["ms_update"] - band_ms
    upd_ms_launch = upd_ms_total / launches
    sieve_ms_launch = seq["ms_sieve"] / seq["sieve_launches"]
    k_upd = seq["k_quotients"] - band_q  # explicit-k pairs k_update takes
    quot = seq["rl_quotients"] + k_upd
    upd_tops = quot / launches * OPS_PER_QUOTIENT / (upd_ms_launch * 1e-3) / 1e12
    # k_update's HBM view: the method's bytes = one int32 M(y) per explicit-k
    # pair (a random read) + the run-length masks (8 bytes per 32 y) read once
    # per 64-x tile over y <= Y; the record-layout view counts the 16-byte
    # record this build reads per explicit-k pair instead
    mask_bytes = 0.25 * seq["sum_Y"] / 64
    upd_bytes = (GATHER_BYTES * k_upd + mask_bytes) / launches
    upd_gbs = upd_bytes / (upd_ms_launch * 1e-3) / 1e9
    rec_bytes = (RECORD_BYTES * k_upd + mask_bytes) / launches
    rec_gbs = rec_bytes / (upd_ms_launch * 1e-3) / 1e9
    # sieve: the records it writes, 0.5 byte per y
    sieve_gbs = (sieved / seq["sieve_launches"]) * 0.5 / (sieve_ms_launch * 1e-3) / 1e9
    upd_view = {"kernel": "k_update", "bound": "alu", "achieved": upd_tops,
                "peak": INT_VALU_PEAK_TOPS, "unit": "TOP/s", "frac": upd_tops / INT_VALU_PEAK_TOPS,
                "traffic": traffic_per_launch("k_update"),
                "ops_rule": (f"{OPS_PER_QUOTIENT} lane-ops per pair (quotient by fused "
                             f"multiply-add with a reciprocal, signed accumulation), run-length "
                             f"pairs + the explicit-k pairs outside the band; peak = 256 CUs x "
                             f"64 lanes x 2.4 GHz"),
                "avg_launch_ms": upd_ms_launch, "launches": launches,
                "pairs_per_launch": quot / launches,
                "hbm_view": {"achieved": upd_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": upd_gbs / HBM_PEAK_GBS, "bytes_per_launch": upd_bytes,
                             "rule": (f"{GATHER_BYTES} B (one int32 M(y)) per explicit-k pair + "
                                      f"8 B of mu masks per 32 y per 64-x tile of the "
                                      f"run-length part")},
                "record_layout_view": {"achieved": rec_gbs, "frac": rec_gbs / HBM_PEAK_GBS,
                                       "bytes_per_launch": rec_bytes,
                                       "rule": f"{RECORD_BYTES} B record per explicit-k pair"}}
    sieve_view = {"kernel": "k_sieve", "bound": "hbm", "achieved": sieve_gbs,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sieve_gbs / HBM_PEAK_GBS,
                  "traffic": traffic_per_launch("k_sieve"), "avg_launch_ms": sieve_ms_launch,
                  "launches": seq["sieve_launches"],
                  "rule": "0.5 B of records written per y (VALU and LDS atomics bound it)"}
    band_view = None
    if band_ms > 0 and band_q > 0:
        band_tops = band_q * OPS_PER_QUOTIENT / (band_ms * 1e-3) / 1e12
        band_view = {"kernel": "k_ek_window", "ms": band_ms, "pairs": band_q,
                     "alu_achieved_TOPs": band_tops,
                     "alu_frac": band_tops / INT_VALU_PEAK_TOPS,
                     "hbm_view_GBs": GATHER_BYTES * band_q / (band_ms * 1e-3) / 1e9,
                     "rule": (f"{OPS_PER_QUOTIENT} lane-ops and {GATHER_BYTES} B per explicit-k "
                              f"pair whose M(y) read lies in the band (records staged in LDS)")}
    if upd_ms_total >= seq["ms_sieve"]:
        roof = dict(upd_view)
        roof["others"] = {"k_sieve": sieve_view, "k_ek_window": band_view}
    else:
        roof = dict(sieve_view)
        roof["others"] = {"k_update": upd_view, "k_ek_window": band_view}
    roof["traffic_unit"] = ("bytes per launch between L2 and memory (rocprofv3 FETCH_SIZE x2 + "
                            "WRITE_SIZE x1, calibrated on a plain copy)")
    roof["in_turn_ms"] = {k: seq[k] for k in ("ms_sieve", "ms_prep", "ms_update", "ms_band",
                                               "ms_total")}
    line = {
        "metric": METRIC,
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
        "quotients": {"run_length": st["rl_quotients"], "explicit_k": st["k_quotients"],
                      "explicit_k_band": st["band_quotients"]},
        "roofline": roof,
    }
    # the byproduct M(10^16 // 10^4) = M(10^12), checked against the oracle
    line["byproduct_1e12"] = int(mt.byproducts(0, 10**4)[10**4 - 1])
    line["tuning"] = mt.tuning()
    if not args.no_batched:
        progress("batched workload: 258 n, one at a time and as one sweep")
        line["batched"] = dict(batched_workload(mt), workload=BATCHED_WORKLOAD)
    return line


BATCHED_WORKLOAD = ("256 n log-uniform in [1e13, 1e17] (seed 0) + 1e16 + 1e17: one shared "
                    "sweep (automatic u) vs each n alone")


def batched_workload(mt) -> dict:
    """The batched workload as one shared sweep against one query at a time;
    Table 1 pins two members."""
    from paper_1108_0135_amd import inputs
    ns = [int(v) for v in inputs.batch_log_uniform(seed=0, count=256, lo=1e13, hi=1e17)]
    ns += [10**16, 10**17]
    res = batched_vs_plain(mt, ns)
    if res["results"][-2] != inputs.TABLE1[10**16] or res["results"][-1] != inputs.TABLE1[10**17]:
        raise RuntimeError("batched Table 1 values wrong")
    del res["results"]
    return res


def workload_batched(args, mt) -> dict:
    res = batched_workload(mt)
    return {"metric": METRIC, "value": res["batched_qps"], "unit": "queries/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": BATCHED_WORKLOAD}, "tuning": mt.tuning(), **res}


def _serve_trace(mt, times, ns):
    """Submit each n at its arrival time, poll until every result is in;
    returns (results, latencies, makespan)."""
    mt.init(0, 0)
    t_base = time.perf_counter()
    pending, lat, got = {}, [0.0] * len(ns), [None] * len(ns)
    i = 0
    while i < len(ns) or pending:
        now = time.perf_counter() - t_base
        while i < len(ns) and times[i] <= now:
            t = mt.submit(ns[i])
            if t is None:
                break
            pending[t] = i
            i += 1
        for t in list(pending):
            r = mt.poll(t)
            if r is not None:
                j = pending.pop(t)
                got[j], lat[j] = r
        time.sleep(0.001)
    makespan = time.perf_counter() - t_base
    mt.shutdown()
    return got, lat, makespan


def workload_serving(args, mt) -> dict:
    """Poisson arrivals at each rate of --rates (the same --count values of n,
    log-uniform in [1e10, 1e18], seed 0) through mertens_submit/poll, against
    a one-at-a-time FIFO server whose service times are each n's measured
    time alone.  Results must equal the one-at-a-time values."""
    import numpy as np
    from paper_1108_0135_amd import inputs
    rates = [float(r) for r in args.rates.split(",")]
    _, ns0 = inputs.poisson_trace(seed=0, rate=rates[0], count=args.count)
    ns = [int(v) for v in ns0]
    progress(f"serving: {len(ns)} values of n one at a time (FIFO service times)")
    mt.init(0, 0)
    mt.query([10**12])
    service, ref = [], []
    for k, n in enumerate(ns):
        t0 = time.perf_counter()
        ref.append(int(mt.query([n])[0]))
        service.append(time.perf_counter() - t0)
        if k % 25 == 24:
            progress(f"one at a time: {k + 1} of {len(ns)}")
    mt.shutdown()
    p = lambda v, q: float(np.percentile(v, q))
    sweep = []
    for rate in rates:
        times, ns_r = inputs.poisson_trace(seed=0, rate=rate, count=args.count)
        if [int(v) for v in ns_r] != ns:
            raise RuntimeError("the trace's n depend on the rate")
        finish, fifo_lat = 0.0, []
        for a_t, s_t in zip(times, service):
            start = max(a_t, finish)
            finish = start + s_t
            fifo_lat.append(finish - a_t)
        fifo_makespan = finish - times[0]
        progress(f"serving at {rate:g} q/s")
        got, lat, makespan = _serve_trace(mt, times, ns)
        if got != ref:
            raise RuntimeError(f"served results differ from one-at-a-time results at {rate} q/s")
        sweep.append({"rate": rate,
                      "served": {"qps": len(ns) / makespan, "p50_s": p(lat, 50),
                                 "p99_s": p(lat, 99)},
                      "fifo_plain": {"qps": len(ns) / fifo_makespan, "p50_s": p(fifo_lat, 50),
                                     "p99_s": p(fifo_lat, 99)}})
    best = max(sweep, key=lambda r: r["served"]["qps"])
    return {"metric": METRIC, "value": best["served"]["qps"], "unit": "queries/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"Poisson arrivals at {args.rates} q/s, {args.count} queries each, "
                                   "n log-uniform in [1e10,1e18], seed 0",
                       "parallelism": "1 GPU"},
            "one_at_a_time_total_s": float(sum(service)), "sweep": sweep}


IV_WIDTH = 2**35  # interval workload: [EXTREME_N, EXTREME_N + 2^35]


def cpu_baseline_interval() -> dict:
    """The oracle's interval tier (O3) on a 2^21-wide piece of the same interval."""
    import oracle
    from paper_1108_0135_amd import inputs
    oracle.build()
    w = 2**21
    t0 = time.perf_counter()
    r = oracle.interval(inputs.EXTREME_N, inputs.EXTREME_N + w, inputs.EXTREME_M)
    dt = time.perf_counter() - t0
    if (r["n_min"], r["m_min"]) != (inputs.EXTREME_N, inputs.EXTREME_M):
        raise RuntimeError("oracle interval missed the Section 6 extreme")
    return {"value": (w + 1) / dt, "unit": "y/s", "cores": 1, "kind": "oracle",
            "sample": f"O3 over [{inputs.EXTREME_N}, +2^21] (single thread, {dt:.1f} s, most of "
                      f"it building its prime table up to 3.4e9)"}


def workload_interval(args, mt) -> dict:
    """Section 6 localization: every M(n) over a 2^35-wide interval starting at the
    printed extreme, from its printed value, and the extremes of M(n)/sqrt(n)."""
    import torch
    from paper_1108_0135_amd import inputs
    a, b = inputs.EXTREME_N, inputs.EXTREME_N + IV_WIDTH
    mt.init(0, 0)

    def step():
        r = mt.interval(a, b, m_a=inputs.EXTREME_M)
        if (r["n_min"], r["m_min"]) != (inputs.EXTREME_N, inputs.EXTREME_M):
            raise RuntimeError(f"interval minimum moved: {r}")
        return r, mt.stats()

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [step()[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_step = 1000.0 * (time.perf_counter() - t0) / args.steps
    st = sts[-1]
    avg = lambda k: sum(x[k] for x in sts) / len(sts)
    # per-kernel launch times (HIP events on the library stream) and
    # algorithmic bytes: the fill pass writes one 4-byte entry per multiple of
    # a bucketed prime and reads each bucketed prime's 8-byte {p, residue};
    # the regrouping pass reads and writes every entry once; the sieve reads
    # its entries and writes 0.5 byte of records per y
    nb = st["blocks"]
    ent = st["bucket_entries"] / nb
    kern = {
        "k_bucket_regroup": (st["ms_bucket_regroup"] / nb, 8 * ent),
        "k_prime_buckets_fill": (st["ms_bucket_fill"] / nb, 4 * ent + 8 * st["bucket_prime_visits"] / nb),
        "k_sieve": (st["ms_sieve"] / nb, 4 * ent + 0.5 * st["sieved_y"] / nb),
    }
    name = max(kern, key=lambda k: kern[k][0])
    ms_l, bytes_l = kern[name]
    gbs = bytes_l / (ms_l * 1e-3) / 1e9
    roof = {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic_per_launch(name, "interval1e19"),
            "algorithmic_bytes_per_launch": bytes_l, "avg_launch_ms": ms_l, "launches": nb,
            "entries_per_launch": ent,
            "traffic_unit": ("bytes per launch between L2 and memory (rocprofv3 FETCH_SIZE x2 + "
                             "WRITE_SIZE x1, calibrated on a plain copy)"),
            "per_kernel_ms": {k: v[0] for k, v in kern.items()}}
    return {
        "metric": "values of M(n) per second over an interval (Section 6 localization)",
        "value": (b - a + 1) / (ms_step * 1e-3), "unit": "y/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"interval [11609864264058592345, +2^35] from the printed M there, "
                               f"primes to 3.4e9 (bucketed), y-blocks of 2^31",
                   "blocks": st["blocks"], "parallelism": "1 GPU"},
        "kernel_ms": {k: avg(k) for k in ("ms_prep", "ms_sieve", "ms_update", "ms_bucket_fill",
                                          "ms_bucket_regroup", "ms_total")},
        "roofline": roof,
    }


def workload_window(args, mt) -> dict:
    """The dense window: 1024 n_i = n0 + 997 i (n0 seeded in [1e18, 1.8e19]) as
    one shared sweep (one keyed group of the distinct (x, floor(n_i/x))),
    against the first member alone.  The first eight members' differences
    are the oracle's (stored expected values); member 0 must equal its
    value alone."""
    import torch
    from paper_1108_0135_amd import inputs
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "golden.json")))["window1e19_diffs"]
    ns = [int(v) for v in inputs.dense_window(seed=0, count=1024)]
    if ns[:8] != gold["n"]:
        raise RuntimeError("window inputs differ from the stored ones")
    mt.init(0, 0)
    # a line every 64 blocks on stderr, and per 2^26-y window of block 0
    # (which holds most of the work)
    mt.set_param("progress", 64)
    mt.set_param("update_window", 26)
    progress("dense window: member 0 alone")
    t0 = time.perf_counter()
    alone = int(mt.query([ns[0]])[0])
    t_alone = time.perf_counter() - t0
    st_alone = mt.stats()
    progress(f"dense window: 1024 members, one sweep (member 0 alone took {t_alone:.1f} s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = [int(v) for v in mt.query(ns)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = mt.stats()
    if got[0] != alone or [got[i + 1] - got[i] for i in range(7)] != gold["diffs"]:
        raise RuntimeError("dense window results wrong")
    return {"metric": METRIC, "value": len(ns) / dt, "unit": "queries/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": dt * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "dense window: 1024 n_i = n0 + 997 i, n0 seeded in [1e18, 1.8e19] "
                                   "(seed 0), one shared sweep; first 8 differences against the oracle",
                       "n0": ns[0], "u": st["u"], "blocks": st["blocks"],
                       "entries": st["sum_L"], "parallelism": "1 GPU"},
            "sieved_y_per_s": st["sieved_y"] / dt,
            "pairs": {"run_length": st["rl_quotients"], "explicit_k": st["k_quotients"]},
            "pairs_per_s": (st["rl_quotients"] + st["k_quotients"]) / dt,
            "member0_alone_s": t_alone, "member0_alone_blocks": st_alone["blocks"],
            "one_at_a_time_s_estimated": 1024 * t_alone,
            "speedup_vs_one_at_a_time_estimated": 1024 * t_alone / dt,
            "kernel_ms": {k: st[k] for k in ("ms_sieve", "ms_prep", "ms_update", "ms_finalize",
                                             "ms_total")},
            "tuning": mt.tuning()}


def workload_wide(args, mt) -> dict:
    """M(10^20) through mertens_query_wide (Table 1), one query per step."""
    import torch
    from paper_1108_0135_amd import inputs
    n = 10**20
    mt.init(0, 0)

    def step():
        got = int(mt.query_wide([n])[0])
        if got != inputs.TABLE1[n]:
            raise RuntimeError(f"wrong result M(1e20) = {got}")
        return mt.stats()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_step = 1000.0 * (time.perf_counter() - t0) / args.steps
    st = sts[-1]
    return {"metric": "sieved y/sec through update, M(10^20) past the 64-bit limit",
            "value": st["sieved_y"] / (ms_step * 1e-3), "unit": "sieved y/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": "single query n=1e20 (mertens_query_wide), automatic u",
                       "u": st["u"], "blocks": st["blocks"], "parallelism": "1 GPU"},
            "kernel_ms": {k: st[k] for k in ("ms_sieve", "ms_prep", "ms_update", "ms_finalize",
                                             "ms_total")}}


def workload_copy(args, mt) -> dict:
    """A plain device copy of known size (calibrates HBM byte counters)."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    return {"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
            "GBps": 2 * nbytes / dt / 1e9}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5; 1 for the wide workload)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warmup steps (default 1; 0 for the wide workload)")
    ap.add_argument("--workload",
                    choices=["default", "batched", "serving", "interval", "wide", "window",
                             "copy"],
                    default="default")
    ap.add_argument("--rates", default="10,30,100,300,1000",
                    help="serving: comma-separated arrival rates (q/s)")
    ap.add_argument("--count", type=int, default=200, help="serving: arrivals per rate")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--in-turn", action="store_true",
                    help="sieve strictly in turn with the update (for per-kernel profiles)")
    args = ap.parse_args()
    long_steps = args.workload == "wide"  # about 100 s per step
    if args.steps is None:
        args.steps = 1 if long_steps else 5
    if args.warmup is None:
        args.warmup = 0 if long_steps else 1
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the sweep has no multi-GPU path",
              file=sys.stderr)
        return 2

    # torch first: it and the library share the HIP runtime library, and
    # torch must be the one that loads it
    import torch  # noqa: F401
    from paper_1108_0135_amd import mertens as mt
    try:
        if args.workload == "default":
            line = workload_default(args, mt)
            if not args.no_cpu_baseline:
                progress("oracle timing on the host")
                line["cpu_baseline"] = cpu_baseline(line["config"]["sieved_y"],
                                                    line["byproduct_1e12"])
        elif args.workload == "batched":
            line = workload_batched(args, mt)
        elif args.workload == "interval":
            line = workload_interval(args, mt)
            if not args.no_cpu_baseline:
                line["cpu_baseline"] = cpu_baseline_interval()
        elif args.workload == "wide":
            line = workload_wide(args, mt)
        elif args.workload == "window":
            line = workload_window(args, mt)
        elif args.workload == "copy":
            line = workload_copy(args, mt)
        else:
            line = workload_serving(args, mt)
    except RuntimeError as e:
        print(str(e), file=sys.stderr)
        return 1
    finally:
        mt.shutdown()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
