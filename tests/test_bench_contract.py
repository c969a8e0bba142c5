"""bench.py pieces that run without a GPU: the refusal of several GPUs, the
per-workload step defaults and the rule that counter-based traffic is only
reported while the kernel sources match the ones it was measured on."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    # a committed summary is used exactly while its hash matches the sources
    for kern, wl in (("k_update", "n1e16"), ("k_sieve", "n1e16"),
                     ("k_bucket_regroup", "interval1e19")):
        path = os.path.join(ROOT, "profiles", f"{kern}_{wl}_traffic.json")
        d = json.load(open(path))
        fresh = d["source_sha256"] == bench.kernel_source_sha256()
        assert bench.traffic_per_launch(kern, wl) == (d["hbm_bytes_per_launch"] if fresh else None)
    # a summary taken on other sources is ignored
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_update_n1e16_traffic.json").write_text(
        json.dumps({"source_sha256": "0" * 64, "hbm_bytes_per_launch": 1.0}))
    real = bench.kernel_source_sha256()
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: real)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_per_launch("k_update") is None
    assert bench.traffic_per_launch("k_sieve") is None  # no summary at all
