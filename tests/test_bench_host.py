"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline record built from
per-family event totals, the traffic lookup keyed by the kernel source's hash, the truncation
summary, and the CPU-oracle baseline record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _fam(launches, ms, flops=0.0, byts=0.0):
    return {"launches": launches, "ms": ms, "flops": flops, "bytes": byts}


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_roofline_family_prefers_long_or_stamped_launches():
    prof = {"pchol": _fam(20000, 200.0), "tri_reduce": _fam(700, 150.0), "other": _fam(5000, 40.0),
            "tri_back": _fam(700, 50.0)}
    # pchol averages 10 us per launch (below the long-launch limit for a bracketed family), so
    # tri_reduce wins
    assert bench.roofline_family(prof) == "tri_reduce"
    # the GEMM kernels carry their own stamps: a short average is still kernel time
    stamped = dict(prof, gemm=_fam(20000, 180.0))
    assert bench.roofline_family(stamped) == "gemm"
    # with no eligible family the largest total wins
    short = {"pchol": _fam(20000, 200.0), "other": _fam(5000, 40.0)}
    assert bench.roofline_family(short) == "pchol"


def test_roofline_record_fields_and_fraction():
    prof = {"gemm": _fam(1000, 10.0, flops=8e11), "tri_reduce": _fam(100, 40.0, flops=1e9, byts=4e7)}
    rf = bench.roofline_of(prof, "gemm", fp64=True)
    assert rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s"
    assert rf["peak"] == bench.PEAK["fp64_mfma"]
    # 8e8 flop per launch in 10 us = 80 TFLOP/s
    assert abs(rf["achieved"] - 80.0) < 1e-9
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-15
    rf = bench.roofline_of(prof, "tri_reduce", fp64=True)
    assert rf["bound"] == "alu" and rf["workgroups"] == 1
    assert abs(rf["frac_of_one_cu"] - rf["achieved"] / (rf["peak"] / 256.0)) < 1e-12
    for key in ("achieved", "peak", "unit", "frac", "traffic", "launches", "avg_launch_us"):
        assert key in rf


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    entry = dict(bench.TRAFFIC["tri_reduce"])
    src = os.path.join(ROOT, entry["source"])
    import hashlib
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    monkeypatch.setitem(bench.TRAFFIC, "tri_reduce", dict(entry, sha256_16=h))
    assert bench._traffic("tri_reduce") == entry["bytes_per_launch"]
    monkeypatch.setitem(bench.TRAFFIC, "tri_reduce", dict(entry, sha256_16="0" * 16))
    assert bench._traffic("tri_reduce") is None
    assert bench._traffic("eig_small") is None    # no entry: never measured


def test_truncation_summary():
    infos = [
        {"discarded_weight": 0.0, "trace_before": 1.0, "trace_after": 1.0, "xi_before": 0.5,
         "xi_after": 0.5, "ppt_feasible": 1},
        {"discarded_weight": 1e-3, "trace_before": 1.0, "trace_after": 0.999, "xi_before": 0.5,
         "xi_after": 0.5 * (1 + 1e-9), "ppt_feasible": 1},
        {"discarded_weight": 2e-3, "trace_before": 2.0, "trace_after": 2.002, "xi_before": 0.25,
         "xi_after": 0.25, "ppt_feasible": 0},
    ]
    s = bench._truncation_summary(infos, {"trace": complex(0.998, 0.0)})
    assert s["updates"] == 3 and s["updates_truncated"] == 2
    assert abs(s["discarded_weight_sum"] - 3e-3) < 1e-15
    assert s["discarded_weight_max"] == 2e-3
    assert abs(s["trace_drift_per_update_max"] - 1e-3) < 1e-12
    assert abs(s["trace_drift_circuit"] - 2e-3) < 1e-12
    assert abs(s["xi_rel_change_per_update_max"] - 1e-9) < 1e-15
    assert s["ppt_infeasible"] == 1
    json.dumps(s)


def test_cpu_baseline_record_on_a_small_circuit():
    pytest.importorskip("numpy")
    from workloads import config_m0
    spec = config_m0(0)
    rec = bench._cpu_baseline(spec, 2.0, small_specs=(("m0", spec),))
    assert rec["kind"] == "oracle" and rec["unit"] == "two-site updates/s"
    assert rec["value"] > 0.0 and rec["cores"] >= 1
    assert isinstance(rec["sample"], str) and rec["sample"]
    assert isinstance(rec["blas"], str)
    assert rec["single_thread"].get("cores", 1) == 1
    assert rec["full_circuits"]["m0"]["two_site_updates"] == spec.n_two_site_updates()
    json.dumps(rec)
