"""Roofline bookkeeping of bench.py (host arithmetic only)."""
import importlib.util
import os

import numpy as np
import pytest

_spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)

# the full-size plain FP32 workload: 133.3 M edges, 2.55 M hits, hidden 64
E, N, H = 133_322_378, 2_548_234, 64


@pytest.mark.parametrize("stage", ["edge_step", "edge_step_final"])
def test_edge_step_fraction_is_priced_on_executed_products(stage):
    """A launch that runs exactly at the FP32 matrix peak on the products the
    factorised edge step executes (4H^2 per edge, +2H^2 for the classifier)
    reports frac 1; no physical launch time gives more."""
    x = E * (4 * H * H + (2 * H * H if stage == "edge_step_final" else 0))
    t_peak = x / (157.3e12)
    r = bench.stage_roofline(stage, t_peak * 1e3, 1, E, N, H, "f32", False)
    assert r["bound"] == "mfma"
    assert r["frac"] == pytest.approx(1.0, rel=1e-12)
    # the unfactorised network would need twice (edge step) the products: reported apart, not as frac
    assert r["algorithmic_equivalent_tflops"] > r["achieved"]
    # the measured launch time of the round's kernel trace (23.7 ms) is well below peak
    r = bench.stage_roofline(stage, 23.70, 1, E, N, H, "f32", False)
    assert 0 < r["frac"] < 1


def test_hbm_stage_fractions():
    stages = {"radius_count": {"ms": 4.0, "launches": 1}, "scan": {"ms": 0.05, "launches": 1},
              "radius_emit": {"ms": 0.4, "launches": 1}, "edge_encode": {"ms": 16.0, "launches": 1},
              "compact": {"ms": 0.6, "launches": 1}, "segsum": {"ms": 60.0, "launches": 8}}
    h = bench.stage_hbm(stages, E, E, E // 2, N, 12, H, 4)
    assert h["a6_segsum"]["bytes"] == E * (H * 4 + 4) + N * (2 * H * 4 + 16)
    assert h["a6_segsum"]["ms"] == pytest.approx(7.5)
    assert h["a5_edge_encode"]["bytes"] == E * (H * 4 + 8) + N * 3 * H * 4
    for v in h.values():
        assert 0 < v["frac"] < 1


def test_prefilter_fallback_band():
    from paper_2508_07423_amd.prefilter_train import fallback_band
    kept = np.array([70, 0, 80, 75, 60])
    cand = np.array([100, 0, 100, 100, 100])       # the empty event does not count
    lo, hi = fallback_band(kept, cand, quantile=0.0, margin=0.8)
    assert hi == 1.0 and lo == pytest.approx(0.8 * 0.6)
    assert fallback_band(np.zeros(3), np.zeros(3)) == (0.0, 1.0)


def test_measured_traffic_only_for_the_profiled_source(monkeypatch):
    """The roofline's counter-measured traffic is reported only while the
    kernel's source hashes to what was profiled; a changed source gives null,
    and so does a kernel or workload with no record."""
    import json
    import os
    path = os.path.join(os.path.dirname(bench.__file__), "profiles", "traffic.json")
    rec = next(r for r in json.load(open(path))["records"] if r["kernel"] == "edge_step" and r["dtype"] == "f32")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: rec["source_sha256"])
    assert bench.measured_traffic("edge_step", "c2", "f32") == rec["bytes_per_launch"]
    assert rec["bytes_per_launch"] == rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: "0" * 64)
    assert bench.measured_traffic("edge_step", "c2", "f32") is None
    assert bench.measured_traffic("edge_step", "c9", "f32") is None
