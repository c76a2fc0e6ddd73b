"""Host-side logic of bench.py (no GPU): the HBM traffic summary written from
rocprofv3 counter files and read back for the roofline, and the one-GPU
guard of the command line."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_counters(path, counter, copy_kib, kernel_kib, threads=1024, matrix_cores=True):
    """A counter_collection file shaped like rocprofv3's: the 1 GiB calibration
    copy, two dispatches of the chi2+grad kernel and, with matrix cores, one
    matrix-core kernel."""
    rows = [("__amd_rocclr_copyBuffer", 131072, copy_kib)]
    for v in kernel_kib:
        rows.append((f"void rime::rime_main<float, {threads}, 2, 32, 2, false>(rime::KParams)",
                     6400, v))
    if matrix_cores:
        rows.append(("rime::pme_forward(rime::KParams)", 25600, 123.0))
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, val) in enumerate(rows):
            r = {k: 0 for k in FIELDS}
            r.update({"Dispatch_Id": i + 1, "Grid_Size": grid, "Kernel_Name": name,
                      "Counter_Name": counter, "Counter_Value": val})
            w.writerow(r)


def test_traffic_round_trip(tmp_path):
    fetch4, write4 = tmp_path / "f4.csv", tmp_path / "w4.csv"
    fetch5, write5 = tmp_path / "f5.csv", tmp_path / "w5.csv"
    # the copy reads half its bytes on FETCH_SIZE (factor 2) and all on WRITE_SIZE
    write_counters(fetch4, "FETCH_SIZE", 524288.0, [1000.0, 1100.0])
    write_counters(write4, "WRITE_SIZE", 1048576.0, [300.0, 300.0])
    write_counters(fetch5, "FETCH_SIZE", 524288.0, [500.0, 500.0], threads=256)
    write_counters(write5, "WRITE_SIZE", 1048576.0, [200.0, 200.0], threads=256)
    out = tmp_path / "traffic.json"
    bench.write_traffic([(str(fetch4), str(write4)), (str(fetch5), str(write5))], str(out))
    tr = json.loads(out.read_text())
    assert tr["kernel_source_sha256"] == bench.kernel_source_digest()
    e4, e5 = tr["entries"]
    assert e4["variant"] == [1024, 2, 32, 1] and e5["variant"] == [256, 2, 32, 1]
    assert e4["fetch_scale"] == pytest.approx(2.0) and e4["write_scale"] == pytest.approx(1.0)
    assert e4["grad_mixed_bytes_per_launch"] == pytest.approx((1050.0 * 2 + 300.0) * 1024)
    assert e5["grad_mixed_bytes_per_launch"] == pytest.approx((500.0 * 2 + 200.0) * 1024)
    # read back: matching variant and workload only
    assert bench.measured_traffic(str(out), [1024, 2, 32, 1], "c2") == pytest.approx(
        e4["grad_mixed_bytes_per_launch"])
    assert bench.measured_traffic(str(out), [256, 2, 32, 1], "c2") == pytest.approx(
        e5["grad_mixed_bytes_per_launch"])
    assert bench.measured_traffic(str(out), [256, 2, 32, 0], "c2") is None
    assert bench.measured_traffic(str(out), [1024, 2, 32, 1], "c4") is None
    # a second workload is merged in; the c2 entries stay
    fetch6, write6 = tmp_path / "f6.csv", tmp_path / "w6.csv"
    write_counters(fetch6, "FETCH_SIZE", 524288.0, [700.0], threads=256)
    write_counters(write6, "WRITE_SIZE", 1048576.0, [100.0], threads=256)
    bench.write_traffic([(str(fetch6), str(write6))], str(out), "c4")
    assert bench.measured_traffic(str(out), [256, 2, 32, 1], "c4") == pytest.approx(
        (700.0 * 2 + 100.0) * 1024)
    assert bench.measured_traffic(str(out), [256, 2, 32, 1], "c2") == pytest.approx(
        e5["grad_mixed_bytes_per_launch"])
    tr = json.loads(out.read_text())
    assert len(tr["entries"]) == 3
    # another kernel source: the summary no longer applies
    tr["kernel_source_sha256"] = "0" * 64
    out.write_text(json.dumps(tr))
    assert bench.measured_traffic(str(out), [1024, 2, 32, 1], "c2") is None
    assert bench.measured_traffic(str(tmp_path / "missing.json"), [1024, 2, 32, 1], "c2") is None


def test_traffic_rejects_mixed_variants(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fetch, "FETCH_SIZE", 524288.0, [1000.0])
    write_counters(write, "WRITE_SIZE", 1048576.0, [300.0], threads=256)
    with pytest.raises(SystemExit):
        bench.write_traffic([(str(fetch), str(write))], str(tmp_path / "t.json"))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
