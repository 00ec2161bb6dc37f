"""Host logic of bench.py (no GPU): the committed counter summaries parse,
figures taken on other force-kernel sources are refused, the FLOP rate is
scaled as documented, and a multi-GPU request exits before touching a GPU."""
import os
import subprocess
import sys

import pytest

import bench


def _summary(path):
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


@pytest.mark.parametrize("path,keys", [
    (bench.TRAFFIC_FILE, ["hbm_bytes_per_launch", "hbm_bytes_per_launch_energy", "fetch_factor",
                          "write_factor"]),
    (bench.FLOPS_FILE, ["fp32_flops_per_launch", "fp32_trans_per_launch", "fp64_flops_per_launch",
                        "fp64_trans_per_launch", "valu_insts_per_entry", "entries_per_launch"]),
])
def test_counter_summaries_parse(path, keys):
    kv = _summary(path)
    assert len(kv.get("force_source_sha256_16", "")) == 16
    for k in keys:
        assert float(kv[k]) >= 0.0, k
    text = open(path).read()
    assert "rocprofv3 --pmc" in text and "bench.py" in text  # the command that made it


def test_summaries_refused_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "force_src_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None
    assert bench.measured_flops(1e-4, 7.5e7) is None


def test_flop_rate_scaling(monkeypatch):
    kv = _summary(bench.FLOPS_FILE)
    monkeypatch.setattr(bench, "force_src_hash", lambda: kv["force_source_sha256_16"])
    avg_s, entries = 1e-4, 7.5e7
    f = bench.measured_flops(avg_s, entries)
    k = entries / float(kv["entries_per_launch"])
    f32 = float(kv["fp32_flops_per_launch"]) + float(kv["fp32_trans_per_launch"])
    f64 = float(kv["fp64_flops_per_launch"]) + float(kv["fp64_trans_per_launch"])
    assert f["fp32_tflops"] == pytest.approx(f32 * k / avg_s / 1e12)
    assert f["fp64_tflops"] == pytest.approx(f64 * k / avg_s / 1e12)
    assert f["frac_fp32"] == pytest.approx(f["fp32_tflops"] / 157.3)
    assert f["frac_fp64"] == pytest.approx(f["fp64_tflops"] / 78.6)
    issue = float(kv["valu_insts_per_entry"]) * entries / avg_s / (256 * 64 * 2.4e9)
    assert f["valu_issue_frac"] == pytest.approx(issue)


def test_traffic_read_when_sources_match(monkeypatch):
    kv = _summary(bench.TRAFFIC_FILE)
    monkeypatch.setattr(bench, "force_src_hash", lambda: kv["force_source_sha256_16"])
    assert bench.measured_traffic() == pytest.approx(float(kv["hbm_bytes_per_launch"]))


def test_multi_gpu_request_exits():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
