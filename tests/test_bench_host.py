"""Host logic of bench.py (no GPU): the one-GPU gate, the HBM-traffic
ingestion from rocprofv3 counter collections (calibrated by a plain device
copy of known size) and the lookup of that record, which is valid only for
the kernel sources it was measured on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COLS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            r = {c: 0 for c in COLS}
            r.update(Correlation_Id=i + 1, Dispatch_Id=i + 1, Agent_Id="Agent 1", Grid_Size=grid,
                     Kernel_Name=name, Workgroup_Size=256, Counter_Name=counter, Counter_Value=value)
            w.writerow(r)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_ingest_counters_scales_by_the_copy_and_picks_the_full_batch_dispatch(tmp_path, monkeypatch):
    """A 1 GiB copy that FETCH_SIZE reports as 512 MiB (factor 2) and
    WRITE_SIZE as 1 GiB (factor 1); a kernel's record is its largest-grid
    dispatch, the first one of that grid."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "csrc_hash", lambda: "h0")
    (tmp_path / "profiles").mkdir()
    gib = 1 << 30
    fetch = [("__amd_rocclr_copyBuffer", 65536, gib / 2 / 1024),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 64 * 256, 10.0),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 2048 * 256, 1000.0),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 2048 * 256, 999.0),
             ("void rs::mf::kf_leaf_up<float, 32, 16>(rs::GroupArgs)", 2048 * 256, 500.0)]
    write = [("__amd_rocclr_copyBuffer", 65536, gib / 1024),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 64 * 256, 1.0),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 2048 * 256, 300.0),
             ("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 2048 * 256, 301.0),
             ("void rs::mf::kf_leaf_up<float, 32, 16>(rs::GroupArgs)", 2048 * 256, 200.0)]
    _csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), gib, "wl")
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))
    by = {r["kernel"]: r for r in rec["records"]}
    assert set(by) == {"km_leaf_up", "kf_leaf_up"}
    km, kf = by["km_leaf_up"], by["kf_leaf_up"]
    assert km["workload"] == "wl_fp64" and kf["workload"] == "wl_mixed"
    assert km["fetch_scale"] == pytest.approx(2.0) and km["write_scale"] == pytest.approx(1.0)
    assert km["bytes_per_launch"] == pytest.approx(1000.0 * 1024 * 2 + 300.0 * 1024)
    assert kf["bytes_per_launch"] == pytest.approx(500.0 * 1024 * 2 + 200.0 * 1024)
    # valid only for the sources it was measured on
    assert bench.load_traffic("km_leaf_up", "wl_fp64") == pytest.approx(km["bytes_per_launch"])
    assert bench.load_traffic("km_leaf_up", "wl_mixed") is None
    monkeypatch.setattr(bench, "csrc_hash", lambda: "h1")
    assert bench.load_traffic("km_leaf_up", "wl_fp64") is None


def test_ingest_counters_without_a_copy_dispatch_fails(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    rows = [("void rs::mf::km_leaf_up<32, 16>(rs::GroupArgs)", 2048 * 256, 1000.0)]
    _csv(tmp_path / "f.csv", "FETCH_SIZE", rows)
    _csv(tmp_path / "w.csv", "WRITE_SIZE", rows)
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1 << 30, "wl")
    assert not (tmp_path / "profiles" / "traffic.json").exists()
