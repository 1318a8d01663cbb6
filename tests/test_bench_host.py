"""Host logic of bench.py (no GPU): counter summaries, the calibration that
turns FETCH_SIZE / WRITE_SIZE into HBM bytes, kernel-name mapping, the
source-hash gate on recorded traffic, and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEMM = "void symten::gemm_f32_kernel<symten::ArgPtrs, symten::TileShape<64, 64, 32> >(symten::TileWork const*, x)"
COPY = "void symten::copy_kernel<symten::ArgPtrs, float, 3>(symten::CopyTask const*, long const*, int, x)"
CAL = "__amd_rocclr_copyBuffer"


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_profile_names():
    assert bench.profile_name(GEMM) == "gemm_f32_kernel<64x64x32,f32>"
    assert bench.profile_name(COPY) == "copy_kernel<f32,bf16x2>"
    # the bf16 kernel's template arguments after the tile: its number of
    # planes, then whether it has the scatter epilogue
    assert bench.profile_name(
        "void symten::gemm_bf16_kernel<symten::DevPtrs, symten::TileShape<256, 128, 32>, 2, false>(a)") == \
        "gemm_bf16_kernel<256x128x32,bf16x3>"
    assert bench.profile_name(
        "void symten::gemm_bf16_kernel<symten::DevPtrs, symten::TileShape<64, 128, 32>, 2, true>(a)") == \
        "gemm_bf16_kernel<64x128x32,bf16x3,scatter>"
    assert bench.profile_name(
        "void symten::gemm_bf16_kernel<symten::DevPtrs, symten::TileShape<64, 64, 32>, 3, false>(a)") == \
        "gemm_bf16_kernel<64x64x32,bf16x6>"
    assert bench.profile_name(
        "void symten::gemm_bf16_kernel<symten::ArgPtrs, symten::TileShape<64, 64, 32>, 1, false>(a)") == \
        "gemm_bf16_kernel<64x64x32,bf16>"
    assert bench.profile_name(COPY.replace("float, 3>", "float, 5>")) == "copy_kernel<f32,bf16x3>"
    assert bench.profile_name(
        "void symten::gemm_f64_kernel<symten::ArgPtrs, symten::TileShape<64, 128, 32> >(a)") == \
        "gemm_f64_kernel<64x128x32>"
    assert bench.profile_name("void rocsolver::latrd_kernel<double>(int)") is None


def test_pmc_summary_averages_per_dispatch(tmp_path):
    # a counter split over two rows of one dispatch (two XCD instances) is summed
    _counter_csv(str(tmp_path / "a"), [
        {"Dispatch_Id": 1, "Kernel_Name": GEMM, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
        {"Dispatch_Id": 1, "Kernel_Name": GEMM, "Counter_Name": "FETCH_SIZE", "Counter_Value": 50},
        {"Dispatch_Id": 2, "Kernel_Name": GEMM, "Counter_Name": "FETCH_SIZE", "Counter_Value": 250},
    ])
    out = bench.pmc_summary(str(tmp_path / "a"))
    assert out == [{"kernel": GEMM, "counter": "FETCH_SIZE", "dispatches": 2, "avg_per_dispatch": 200.0}]


def test_write_traffic_scales_by_the_calibration_copy(tmp_path):
    """FETCH_SIZE reads half a byte per byte of the 256 MiB copy, WRITE_SIZE
    one: a kernel's KiB per dispatch become bytes per launch divided by those
    factors, and its traffic is their sum."""
    mib256 = 256 << 20
    base = tmp_path / "pmc"
    for c, per_byte, kib in (("FETCH_SIZE", 0.5, 3000.0), ("WRITE_SIZE", 1.0, 1000.0)):
        _counter_csv(str(base / ("pmc_copy_" + c)), [
            {"Dispatch_Id": 7, "Kernel_Name": CAL, "Counter_Name": c, "Counter_Value": per_byte * mib256 / 1024}])
        _counter_csv(str(base / ("pmc_" + c)), [
            {"Dispatch_Id": 3, "Kernel_Name": GEMM, "Counter_Name": c, "Counter_Value": kib}])
        for d in ("pmc_copy_" + c, "pmc_" + c):
            json.dump(bench.pmc_summary(str(base / d)), open(str(base / (d + ".summary.json")), "w"))
    out = str(tmp_path / "traffic.json")
    rec = bench.write_traffic(str(base), "w0", "cmd", out=out)
    k = rec["kernels"]["gemm_f32_kernel<64x64x32,f32>"]
    assert rec["calibration"]["fetch_counter_per_byte"] == pytest.approx(0.5)
    assert rec["calibration"]["write_counter_per_byte"] == pytest.approx(1.0)
    assert k["fetch_bytes_per_launch"] == pytest.approx(3000.0 * 1024 / 0.5)
    assert k["write_bytes_per_launch"] == pytest.approx(1000.0 * 1024)
    assert k["bytes_per_launch"] == pytest.approx(3000.0 * 2048 + 1000.0 * 1024)
    assert json.load(open(out)) == rec
    assert rec["sources_sha256"] == bench.sources_sha256()


def test_recorded_traffic_is_gated_by_the_source_hash():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    name = next(iter(rec["kernels"]))
    if rec["sources_sha256"] == bench.sources_sha256():
        assert bench.traffic_for(name, rec["workload"]) == rec["kernels"][name].get("bytes_per_launch")
    else:
        assert bench.traffic_for(name, rec["workload"]) is None
    assert bench.traffic_for(name, "another_workload") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
