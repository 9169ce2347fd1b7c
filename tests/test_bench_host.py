"""Host logic of bench.py (no GPU): the roofline objects, the gating of the recorded HBM
traffic figure, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_fp32_roofline_against_fp32_mfma_peak():
    r = bench.m2l_roofline("fp32", 104.0, 15.35e9)
    assert r["bound"] == "mfma" and r["peak"] == 157.3 and r["unit"] == "TFLOP/s"
    assert r["frac"] == pytest.approx(104.0 / 157.3) and r["traffic"] == 15.35e9
    assert r["traffic_source"].startswith("profiles/") and "L2-to-fabric" in r["traffic_kind"]


def test_mixed_roofline_counts_three_fp16_products():
    r = bench.m2l_roofline("mixed", 89.0, 15.35e9)
    assert r["peak"] == 2500.0 and r["achieved"] == pytest.approx(267.0)
    assert r["fp32_equivalent"] == 89.0 and r["traffic"] == 15.35e9
    assert r["traffic_source"] == bench.M2L_TRAFFIC_MIXED["source"]
    assert bench.m2l_roofline("mixed", 89.0, None)["traffic_source"] is None


def test_p2p_roofline_has_no_ceiling_above_one():
    r = bench.p2p_roofline(47.6)
    assert r["bound"] == "alu" and r["peak"] == 78.6 and r["frac"] == pytest.approx(47.6 / 78.6)
    assert all(not k.startswith("frac") or v <= 1 for k, v in r.items() if isinstance(v, float))


def test_default_workload_is_the_largest_single_gpu_configuration():
    a = bench.parse([])
    assert a.workload == "uniform-16M" and a.precision == "fp32" and a.p is None


def test_traffic_only_for_the_measured_kernel_and_grouping(monkeypatch):
    t = dict(bench.M2L_TRAFFIC, kernel_sha256="ab" * 8, entries=123, work_items=45, bytes=7.5e9)
    monkeypatch.setattr(bench, "M2L_TRAFFIC", t)
    st = {"m2l_entries": t["entries"], "m2l_work_items": t["work_items"]}
    assert len(bench.m2l_kernel_sha()) == 16
    monkeypatch.setattr(bench, "m2l_kernel_sha", lambda mixed=False: t["kernel_sha256"])
    assert bench.m2l_traffic(t["workload"], t["p"], t["theta"], st) == t["bytes"]
    assert bench.m2l_traffic(t["workload"], t["p"], 0.5, st) is None
    assert bench.m2l_traffic("sphere-4M", t["p"], t["theta"], st) is None
    st2 = dict(st, m2l_entries=st["m2l_entries"] + 1)
    assert bench.m2l_traffic(t["workload"], t["p"], t["theta"], st2) is None
    monkeypatch.setattr(bench, "m2l_kernel_sha", lambda mixed=False: "0" * 16)   # the kernel changed since
    assert bench.m2l_traffic(t["workload"], t["p"], t["theta"], st) is None


def test_mixed_traffic_keyed_to_the_mixed_kernel_and_grouping(monkeypatch):
    tm = dict(bench.M2L_TRAFFIC_MIXED, kernel_sha256="cd" * 8, entries=77, work_items=11, bytes=6.5e9)
    monkeypatch.setattr(bench, "M2L_TRAFFIC_MIXED", tm)
    assert len(bench.m2l_kernel_sha(True)) == 16 and bench.m2l_kernel_sha(True) != bench.m2l_kernel_sha()
    monkeypatch.setattr(bench, "m2l_kernel_sha", lambda mixed=False: "cd" * 8 if mixed else "ef" * 8)
    st = {"m2l_entries": 77, "m2l_work_items": 11}
    assert bench.m2l_traffic(tm["workload"], tm["p"], tm["theta"], st, mixed=True) == 6.5e9
    assert bench.m2l_traffic(tm["workload"], tm["p"], tm["theta"], st) is None     # the FP32 record does not match
    assert bench.m2l_traffic(tm["workload"], tm["p"], tm["theta"], dict(st, m2l_work_items=12), mixed=True) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr
