"""Host logic of bench.py that runs without a GPU: the one-GPU refusal, the
traffic figure taken from a committed counter summary only while the kernel
source is the one it was measured on, and the roofline arithmetic."""
import importlib.util
import math
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def write_summary(path, sha, nbytes):
    with open(path, "w") as f:
        f.write("# k_refine, HBM traffic\n\n")
        f.write(f"- `hbm_bytes_per_launch`: `{nbytes}`\n")
        f.write(f"- `kernel_source_sha256`: `{sha}`\n")


def test_traffic_only_for_the_measured_kernel_source(bench, tmp_path, monkeypatch):
    path = tmp_path / "k_refine_traffic_n20000.md"
    monkeypatch.setattr(bench, "traffic_summary", lambda kernel: str(path))
    assert bench.measured_traffic("refine") is None  # no summary
    write_summary(path, bench.kernel_source_sha(), 2.0639e9)
    assert bench.measured_traffic("refine") == 2.0639e9
    write_summary(path, "0" * 64, 2.0639e9)  # kernels changed since the counters were taken
    assert bench.measured_traffic("refine") is None
    write_summary(path, bench.kernel_source_sha(), "n/a")
    assert bench.measured_traffic("refine") is None


def test_committed_traffic_summaries_are_well_formed(bench):
    for kernel in ("refine", "vectors", "vectors_ckpt"):
        path = bench.traffic_summary(kernel)
        assert os.path.exists(path), path
        text = open(path).read()
        sha = re.search(r"`kernel_source_sha256`: `([0-9a-f]+)`", text)
        assert sha and len(sha.group(1)) == 64, path
        val = re.search(r"`hbm_bytes_per_launch`: `([^`]+)`", text)
        assert val and float(val.group(1)) > 0, path


def test_roofline_alu_bound_kernel(bench, monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda kernel: None)
    # 14 launches, 76 ms of events, 2e11 flops of Sturm-count arithmetic
    prof = {"refine": {"ms": 76.0, "launches": 14, "work": 2.0e11, "bytes": 0.0},
            "vectors": {"ms": 41.0, "launches": 1, "work": 0.0, "bytes": 2.1e9},
            "grid": {"ms": 5.0, "launches": 2, "work": 1.9e10, "bytes": 0.0}}
    r = bench.roofline(prof)
    assert r["kernel"] == "refine" and r["symbol"] == "k_refine" and r["bound"] == "alu"
    assert math.isclose(r["avg_ms"], 76.0 / 14)
    assert math.isclose(r["achieved"], 2.0e11 / 0.076 / 1e12)
    assert r["peak"] == 78.6 and r["unit"] == "TFLOP/s"
    assert math.isclose(r["frac"], r["achieved"] / 78.6)
    assert r["traffic"] is None


def test_roofline_hbm_bound_kernel(bench, monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda kernel: 3.0e10)
    prof = {"refine": {"ms": 20.0, "launches": 7, "work": 5e10, "bytes": 0.0},
            "vectors_ckpt": {"ms": 45.0, "launches": 1, "work": 0.0, "bytes": 7.5e9}}
    r = bench.roofline(prof)
    assert r["kernel"] == "vectors_ckpt" and r["symbol"] == "k_vectors" and r["bound"] == "hbm"
    assert math.isclose(r["achieved"], 7.5e9 / 0.045 / 1e9)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert math.isclose(r["frac"], r["achieved"] / 8000.0)
    assert r["traffic"] == 3.0e10
