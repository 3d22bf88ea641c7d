"""Host logic of bench.py that the measurement line rests on (CPU only): the
algorithmic byte model of the push, the HBM traffic record built from two
rocprofv3 counter files, and the refusal of more than one GPU."""

import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_per_particle_and_cell():
    # 2D FP32: read cell 4, two offsets 8, u 12, s 12, w 4; write all but w
    total, per_particle, per_cell = bench.algorithmic_bytes(2, "fp32", 67108864, 4194304)
    assert (per_particle, per_cell) == (76, 36)
    assert total == 5251268608                                    # c2, as the bench line reports
    assert total / 67108864 == pytest.approx(78.25)               # 16 particles per cell
    assert bench.algorithmic_bytes(3, "fp32", 1, 0)[1] == 84
    assert bench.algorithmic_bytes(2, "fp64", 1, 1)[1:] == (144, 72)
    # the FP64 grid the library keeps: 72 B per cell in the FP32 path too
    assert bench.algorithmic_bytes(2, "fp32", 0, 1, grid_bytes=8)[2] == 72
    total3, _, _ = bench.algorithmic_bytes(3, "fp32", 134217728, 33554432)
    assert total3 / 134217728 == pytest.approx(93.0)


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name + "(args)", "Counter_Name": counter,
                        "Counter_Value": value})


@pytest.mark.parametrize("rec_name", ["spinpic::k_push_tiles_rec<float, double, 2>",
                                      "spinpic::k_push_tiles<float, double, 2, true>"])
def test_traffic_record_takes_the_push_without_the_record(tmp_path, monkeypatch, rec_name):
    """The probe calibrates the counters (the copy reads 1 GiB over its
    dispatches, the fill writes 1 GiB); the record is the push without the
    Eq. 4 record, whichever name the kernel that keeps it has."""
    push = "spinpic::k_push_tiles<float, double, 2, false>"
    probe_kib = 1024.0 * 1024.0
    fetch = [("__amd_rocclr_copyBuffer", probe_kib / 4)] * 4 + \
            [(push, 1000.0), (push, 3000.0), (rec_name, 9999.0), ("spinpic::k_insert<float, 2>", 5.0)]
    write = [("void at::native::vectorized_elementwise_kernel<FillFunctor>", probe_kib * 0.5)] + \
            [(push, 500.0), (push, 700.0), (rec_name, 8888.0), ("spinpic::k_insert<float, 2>", 6.0)]
    fcsv, wcsv = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(fcsv, "FETCH_SIZE", fetch)
    _counter_csv(wcsv, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_path", lambda workload, precision: str(out))
    bench.write_traffic(str(fcsv), str(wcsv), "c2", "fp32")
    rec = json.loads(out.read_text())
    assert rec["kernel"] == push
    assert rec["fetch_scale"] == pytest.approx(1.0)     # 4 x 1/4 GiB read = the probe
    assert rec["write_scale"] == pytest.approx(2.0)     # the fill counted half its bytes
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024)
    assert rec["write_bytes_per_launch"] == pytest.approx(600.0 * 1024 * 2.0)
    assert rec["bytes_per_launch"] == pytest.approx(2000.0 * 1024 + 1200.0 * 1024)
    assert rec["source_hash"] == bench.source_hash()
    # a record taken on other kernel sources is not used
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("c2", "fp32", None) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
