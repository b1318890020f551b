"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the counter
summary it assembles from rocprofv3 --pmc output, and when it trusts that
summary (same kernel sources, same grid, same population layout)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_dir(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})
    return path


def test_traffic_assembly_and_validity(tmp_path, monkeypatch):
    n = 4096
    copy_kib = 9 * n * n * 4 / 1024.0
    kern = "d2q9_fused_lds"                     # rocprofv3 --pmc prints bare names
    # FETCH_SIZE reads half the copy's bytes (the factor-2 scale measured on
    # the chip), WRITE_SIZE all of them
    d = [_counter_dir(str(tmp_path / "f"), "FETCH_SIZE", [(kern, 300000.0), (kern, 302000.0),
                                                        ("other_kernel", 1.0)]),
         _counter_dir(str(tmp_path / "w"), "WRITE_SIZE", [(kern, 803000.0)]),
         _counter_dir(str(tmp_path / "cf"), "FETCH_SIZE", [("copy_kernel", copy_kib / 2)]),
         _counter_dir(str(tmp_path / "cw"), "WRITE_SIZE", [("copy_kernel", copy_kib)])]
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    monkeypatch.setattr(bench, "LAYOUT", "rows")
    bench.assemble_traffic(d)
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["read_bytes_per_launch"] == pytest.approx(301000.0 * 1024 * 2)
    assert t["write_bytes_per_launch"] == pytest.approx(803000.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(t["read_bytes_per_launch"] + t["write_bytes_per_launch"])
    assert t["layout"] == "rows" and t["cells"] == n * n
    # trusted only for the same sources, grid and layout
    assert bench.traffic_entry(n * n) == pytest.approx(t["bytes_per_launch"])
    assert bench.traffic_entry(n * n + 1) is None
    monkeypatch.setattr(bench, "LAYOUT", "planes")
    assert bench.traffic_entry(n * n) is None
    monkeypatch.setattr(bench, "LAYOUT", "rows")
    t["kernel_hash"] = "0" * 16
    json.dump(t, open(out, "w"))
    assert bench.traffic_entry(n * n) is None


def test_missing_counters_are_an_error(tmp_path):
    empty = _counter_dir(str(tmp_path / "e"), "FETCH_SIZE", [("other_kernel", 1.0)])
    with pytest.raises(SystemExit):
        bench._pmc_mean(empty, "FETCH_SIZE", bench.FUSED_KERNEL_PREFIX)
