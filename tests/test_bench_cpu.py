"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline
arithmetic and the rule that counter-based traffic is reported only for the
kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_arithmetic():
    rf = bench.roofline("f32", 4096, 4096, 1, 0.05)
    assert rf["algorithmic_bytes_per_launch"] == 2 * 4096 * 4096 * 4
    assert rf["achieved"] == pytest.approx(134217728 / 0.05e-3 / 1e9, abs=0.05)     # rounded to 0.1 GB/s
    assert rf["frac"] == pytest.approx(rf["achieved"] / 8000.0, abs=1e-4)
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert bench.roofline("u8", 10, 20, 3, 1.0)["algorithmic_bytes_per_launch"] == 2 * 10 * 20 * 3


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    rec = {"f32_4096x4096_s8_K3": {"kernel_sha": bench.kernel_source_hash(), "hbm_bytes_per_launch": 123}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["f32_4096x4096_s8_K3"]["kernel_sha"])
    assert bench.traffic_record("f32_4096x4096_s8_K3") == 123
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_record("f32_4096x4096_s8_K3") is None
    assert bench.traffic_record("u8_4096x4096_s8_K3") is None


def test_valu_only_for_the_profiled_sources(tmp_path, monkeypatch):
    """uint8 VALU work comes from the committed counter record of the same
    kernel sources: lane-ops per pixel = instructions x 64 / pixels, busy =
    instructions x 4 cycles / (1024 SIMDs x time x 2.4 GHz)."""
    rec = {"u8_4096x4096_s8_K3": {"kernel_sha": "a" * 16, "valu_insts_per_launch": 1.0e7}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "a" * 16)
    v = bench.valu_record("u8_4096x4096_s8_K3", 0.05, 4096 * 4096)
    assert v["lane_ops_per_px"] == pytest.approx(1.0e7 * 64 / 4096 ** 2, abs=0.01)
    assert v["busy_frac"] == pytest.approx(1.0e7 * 4 / (1024 * 0.05e-3 * 2.4e9), abs=1e-3)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "b" * 16)
    assert bench.valu_record("u8_4096x4096_s8_K3", 0.05, 4096 * 4096) is None


def test_roofline_reports_the_copy_ceiling():
    rf = bench.roofline("f32", 4096, 4096, 1, 0.05, copy_gbs=5000.0)
    assert rf["copy_ceiling"] == 5000.0
    assert rf["frac_of_copy"] == pytest.approx(rf["achieved"] / 5000.0, abs=1e-4)
