"""Host logic of bench.py (no GPU): the one-GPU guard and the conversion of
rocprofv3 counter runs into HBM bytes per launch."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _counter_csv(d, name, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": name, "Counter_Value": v})


def test_write_traffic_scales_by_the_copy(tmp_path, monkeypatch):
    """Each counter is scaled so that the copy kernel reads (and writes)
    exactly COPY_BYTES; launches are averaged per launch shape; a shape seen
    by only one of the two counters is left out; the rates kernel is not
    counted."""
    sys.path.insert(0, ROOT)
    import bench
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    kib = bench.COPY_BYTES / 1024.0
    jac = "void pyjac::tile_kernel<8, 512, 1, true, false>(pyjac::MechDev, long)"
    jac2 = "void pyjac::tile_kernel<16, 1024, 1, true, false>(pyjac::MechDev, long)"
    jac3 = "void pyjac::tile_kernel<4, 256, 1, true, true>(pyjac::MechDev, long)"
    rates = "void pyjac::tile_kernel<64, 1024, 4, false, false>(pyjac::MechDev, long)"
    # FETCH reads half the copy's bytes (scale 2), WRITE all of them (scale 1)
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [(jac, 100.0), (jac, 300.0), (jac2, 7.0), (jac3, 3.0), (rates, 5.0),
                                                ("__amd_rocclr_copyBuffer", kib / 2)])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [(jac, 1000.0), (jac, 1000.0), (jac2, 9.0), (rates, 5.0),
                                                ("__amd_rocclr_copyBuffer", kib)])
    assert bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w")) == 0
    d = json.loads(out.read_text())
    assert d["scale"] == pytest.approx({"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0})
    e = d["shapes"]["8x512"]
    assert e["FETCH_SIZE"] == pytest.approx(200.0 * 1024 * 2.0)
    assert e["WRITE_SIZE"] == pytest.approx(1000.0 * 1024)
    assert e["bytes_per_launch"] == pytest.approx(e["FETCH_SIZE"] + e["WRITE_SIZE"])
    assert e["dispatches"] == 2
    assert d["shapes"]["16x1024"]["bytes_per_launch"] == pytest.approx(7.0 * 1024 * 2.0 + 9.0 * 1024)
    assert set(d["shapes"]) == {"8x512", "16x1024"}   # 4x256: FETCH only; rates kernel: not a Jacobian
    assert d["kernel_source_hash"] == bench.kernel_source_hash()
    # a matching hash and shape is reported, anything else is not
    assert bench.measured_traffic((8, 512)) == pytest.approx(e["bytes_per_launch"])
    assert bench.measured_traffic((4, 256)) is None
    assert bench.measured_traffic(None) is None
