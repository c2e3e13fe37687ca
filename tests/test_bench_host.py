"""Host-side accounting of bench.py (no GPU): algorithmic bytes per launch,
the roofline each workload is reported against, and the rule that measured
HBM traffic is reported only for the kernel sources it was measured on."""
import json

import pytest

import bench
from paper_1412_4907_amd import build as pbuild
from paper_1412_4907_amd import synth


def test_algorithmic_bytes_paper_block():
    w = synth.paper()
    x = 1024 * 65536 * 32 * 2                      # int8 voltages, once
    p = 1024 * 128 * (65536 // 16) * 4             # FP32 integrated power, once
    assert bench.algorithmic_bytes(w, "fp32") == x + 1024 * 128 * 32 * 2 * 4 + p
    assert bench.algorithmic_bytes(w, "fp16") == x + 1024 * 128 * 32 * 2 * 2 + p
    w4 = synth.four_bit(w)                         # one byte per antenna sample
    assert bench.algorithmic_bytes(w4, "fp16") == x // 2 + 1024 * 128 * 32 * 2 * 2 + p


def test_roofline_bound_follows_intensity():
    flops = 8.0 * 1024 * 128 * 65536 * 32
    w = synth.paper()
    ab = bench.algorithmic_bytes(w, "fp32")
    r = bench.roofline(140.0, 157.3, ab, 15.7, flops, None)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["frac"] == pytest.approx(140.0 / 157.3, abs=1e-4)
    # the small block (12.8 flop/B) sits below the FP32 ridge (19.7): HBM
    s = synth.small()
    fs = 8.0 * s.n_chan * s.n_beams * s.n_samples * s.n_ant
    r2 = bench.roofline(20.0, 157.3, bench.algorithmic_bytes(s, "fp32"), 0.027, fs, None)
    assert r2["bound"] == "hbm" and r2["unit"] == "GB/s" and r2["peak"] == bench.PEAK_HBM_GBS


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 123.0, "source_hash": pbuild.source_hash()}
    (prof / "traffic.json").write_text(json.dumps({"beamform/paper/fp32": entry}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("beamform/paper/fp32") == 123.0
    assert bench.load_traffic("beamform/other/fp32") is None
    entry["source_hash"] = "0" * 64                # counters from other kernel sources
    (prof / "traffic.json").write_text(json.dumps({"beamform/paper/fp32": entry}))
    assert bench.load_traffic("beamform/paper/fp32") is None
