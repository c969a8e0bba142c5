"""GPU test: mertens_init applies the stored autotuner choice exactly when it
was measured on the kernel sources the library was built from."""
from __future__ import annotations

import json
import os

import pytest

pytestmark = pytest.mark.gpu


def test_tuned_file_applied_only_on_matching_sources(monkeypatch):
    from paper_1108_0135_amd import autotune
    from paper_1108_0135_amd import mertens as mt
    monkeypatch.delenv("MERTENS_TUNED", raising=False)
    path = autotune.TUNED_PATH
    stored = json.load(open(path)) if os.path.exists(path) else {}
    fresh = stored.get("source_sha256") == autotune.kernel_source_sha256()
    mt.init(0, 0)
    try:
        assert mt.get_param("tuned") == (1.0 if fresh else 0.0)
        if fresh:
            for k, v in stored["params"].items():
                assert mt.get_param(k) == pytest.approx(float(v)), k
    finally:
        mt.shutdown()
    # switched off: the built-in defaults
    monkeypatch.setenv("MERTENS_TUNED", "0")
    mt.init(0, 0)
    try:
        assert mt.get_param("tuned") == 0.0
        assert mt.get_param("beta") == 0.25 and mt.get_param("block_auto") == 2**30
    finally:
        mt.shutdown()
