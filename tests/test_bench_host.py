"""CPU-side checks of the benchmark's contract and of its counter ingestion (no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for k, (name, grid, val) in enumerate(rows):
            w.writerow({c: 0 for c in cols} | dict(Correlation_Id=k + 1, Dispatch_Id=k + 1, Grid_Size=grid,
                                                    Kernel_Name=name, Counter_Name=counter, Counter_Value=val))


def test_counter_ingestion_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE records (KiB per dispatch) are scaled by what the same
    counter read for the program's first large copy (4 GiB), launches of the small
    warm-up pair are dropped, and the per-launch bytes land in the traffic record."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "TRAFFIC", str(tmp_path / "traffic.json"))
    kib4g = 4 * 2**20
    col_t = "void fa::k_lse_col_t<4, 8>(float const*, int, int)"
    fetch = [("__amd_rocclr_copyBuffer", 131072, kib4g / 2),          # calibration: read as 2 GiB
             (col_t, 600, 10.0),                                      # warm-up pair: dropped
             (col_t, 3840000, 57.6e9 / 1024 / 2), (col_t, 3840000, 57.6e9 / 1024 / 2),
             ("__amd_rocclr_copyBuffer", 131072, 9e9)]                # a later big copy is not the reference
    write = [("__amd_rocclr_copyBuffer", 131072, kib4g), (col_t, 600, 1.0), (col_t, 3840000, 100.0),
             (col_t, 3840000, 100.0), ("__amd_rocclr_copyBuffer", 131072, 1e9)]
    _write_counters(str(tmp_path / "fetch"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "write"), "WRITE_SIZE", write)
    bench.ingest_counters(str(tmp_path / "fetch"), str(tmp_path / "write"))
    rec = json.load(open(tmp_path / "traffic.json"))
    assert abs(rec["calibration"]["fetch_factor"] - 2.0) < 1e-12 and abs(rec["calibration"]["write_factor"] - 1.0) < 1e-12
    k = rec["kernels"]["lse_col_t"]
    assert k["launches"] == 2
    assert abs(k["fetch_bytes"] - 57.6e9) < 1e3 and abs(k["write_bytes"] - 102400.0) < 1e-6
    assert k["source_digest"] == bench.source_digest("lse_col_t")
