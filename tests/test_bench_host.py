"""Host-side checks of bench.py (no GPU): the one-GPU guard, the HBM traffic
summary built from rocprofv3 csv files, and the source-hash gate that keeps a
stale summary out of the roofline."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERN = "void lt::k_tgemm_bf16<5, 2, 2, 3>(lt::GemmArgs16)"
COPY = "__amd_rocclr_copyBuffer"


def _pmc(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def _trace(path, grids):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"])
        for g in grids:
            w.writerow([KERN, g, 1, 1])


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_prices_full_step_per_work_group(tmp_path):
    """Two sampled grids (1 and 2 launches) and a copy calibration of
    FETCH 2x / WRITE 1x; the full step has 3 launches of grid A, 1 of grid B
    and 1 of a grid the sample lacks (priced at the sample's mean per
    work-group).  Expected bytes computed by hand."""
    gA, gB, gC = 256 * 100, 256 * 50, 256 * 10
    gib_kib = (1 << 30) / 1024
    _pmc(tmp_path / "fetch_counter_collection.csv",
         [(1, gA, KERN, "FETCH_SIZE", 1000.0), (2, gB, KERN, "FETCH_SIZE", 300.0),
          (3, gB, KERN, "FETCH_SIZE", 500.0), (4, 512, "other", "FETCH_SIZE", 9e9)])
    _pmc(tmp_path / "write_counter_collection.csv",
         [(1, gA, KERN, "WRITE_SIZE", 100.0), (2, gB, KERN, "WRITE_SIZE", 40.0),
          (3, gB, KERN, "WRITE_SIZE", 60.0)])
    _pmc(tmp_path / "cfetch_counter_collection.csv", [(1, 512, COPY, "FETCH_SIZE", gib_kib / 2)] * 3)
    _pmc(tmp_path / "cwrite_counter_collection.csv", [(1, 512, COPY, "WRITE_SIZE", gib_kib)] * 3)
    _trace(tmp_path / "trace.csv", [gA, gA, gA, gB, gC])
    out = bench.traffic_from(str(tmp_path), str(tmp_path / "trace.csv"), "bf16x3", "lno",
                             dst=str(tmp_path / "t.json"))
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    # per work-group bytes (KiB * 1024 * scale / work-groups)
    fa, fb = 1000 * 1024 * 2 / 100, 400 * 1024 * 2 / 50
    wa, wb = 100 * 1024 / 100, 50 * 1024 / 50
    fmean = (fa * 100 + fb * 50 * 2) / (100 + 50 * 2)
    wmean = (wa * 100 + wb * 50 * 2) / (100 + 50 * 2)
    fetch = (3 * fa * 100 + fb * 50 + fmean * 10) / 5
    write = (3 * wa * 100 + wb * 50 + wmean * 10) / 5
    assert out["fetch_bytes_per_launch"] == pytest.approx(fetch)
    assert out["write_bytes_per_launch"] == pytest.approx(write)
    assert out["bytes_per_launch"] == pytest.approx(fetch + write)
    assert out["unsampled_grid_launches"] == 1
    assert out["source_hash"] == bench.kernel_source_hash("bf16x3")
    assert json.load(open(tmp_path / "t.json"))["bytes_per_launch"] == pytest.approx(fetch + write)


def test_committed_traffic_is_gated_by_kernel_source_hash(monkeypatch):
    t = bench.committed_traffic("bf16x3", "lno")
    if t is None:
        pytest.skip("no committed traffic summary for the current kernel source")
    assert t["bytes_per_launch"] > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda precision: "0" * 16)
    assert bench.committed_traffic("bf16x3", "lno") is None


COMMON = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
          "scaling", "vs_baseline", "dtype", "data", "config")


def _profiles():
    d = os.path.join(ROOT, "profiles")
    return sorted(os.path.join(d, f) for f in os.listdir(d) if f.startswith("bench_") and f.endswith(".json"))


@pytest.mark.parametrize("path", _profiles(), ids=os.path.basename)
def test_committed_bench_lines_keep_the_contract(path):
    """Every committed bench line carries the contract's keys, names its
    workload, ran on one GPU, and (where it has one) its roofline fraction
    is achieved over peak."""
    with open(path) as f:
        line = json.load(f)
    for k in COMMON:
        assert k in line, k
    assert line["n_gpus"] == 1 and line["steps"] >= 1
    assert "workload" in line["config"] and "model" not in line["config"]
    assert line["data"] == "synthetic" and line["value"] > 0
    r = line.get("roofline")
    if r is not None:
        assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
        assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-4
        assert "traffic" in r


def test_headline_line_has_roofline_traffic_and_cpu_baseline():
    with open(os.path.join(ROOT, "profiles", "bench_bf16x3_lno_domain.json")) as f:
        line = json.load(f)
    r = line["roofline"]
    assert r["peak"] == bench.PEAK_TFLOPS["bf16x3"] and r["traffic"] > 0
    c = line["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
    assert line["parity"]["pass"] is True
