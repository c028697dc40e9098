"""The bench's host-side tools, no GPU: the calibrated traffic figure written from two counter files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": 256, "Counter_Name": counter,
                        "Counter_Value": value})


def test_write_traffic(tmp_path):
    """Dispatches between the source build and the runtime copy are summed and scaled by the copy's factor
    (2 GiB read and written): FETCH_SIZE reads half the bytes on this GPU, WRITE_SIZE all of them."""
    gib2_kib = 2 * 1024 * 1024
    fetch = [("wolf::k_build_source", 64.0), ("wolf::k_slab_half", 1000.0), ("wolf::k_axis_fft", 3000.0),
             ("__amd_rocclr_copyBuffer", gib2_kib / 2), ("wolf::k_sdiag", 5.0)]
    write = [("wolf::k_build_source", 10.0), ("wolf::k_slab_half", 2000.0), ("wolf::k_axis_fft", 6000.0),
             ("__amd_rocclr_copyBuffer", gib2_kib), ("wolf::k_sdiag", 5.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _counter_csv(fp, "FETCH_SIZE", fetch)
    _counter_csv(wp, "WRITE_SIZE", write)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--write-traffic", str(fp), str(wp),
                        "--plan", "3,2048,1024", "--traffic", str(out)], capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    rec = json.load(open(out))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["fetch_bytes"] == int(4000.0 * 1024 * 2.0)
    assert rec["write_bytes"] == int(8000.0 * 1024 * 1.0)
    assert rec["propagate_bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert rec["dispatches"] == 2
    assert rec["plan"] == {"fused_slab": 3, "slab_chunk": 2048, "col_chunk": 1024, "coop_cols": 0,
                           "coop_lookahead": 1}
    assert rec["workload"] == "gsm128_fresnel_c64" and len(rec["kernels_sha"]) == 16


def test_write_traffic_n256_workload(tmp_path):
    """The N = 256 sample's record carries its own workload name and plan, so that the N = 256 roofline and
    the headline each take only their own figure."""
    gib2_kib = 2 * 1024 * 1024
    fetch = [("wolf::k_build_source", 64.0), ("wolf::k_row_fft", 500.0), ("wolf::k_axis_fft", 700.0),
             ("__amd_rocclr_copyBuffer", gib2_kib / 2)]
    write = [("wolf::k_build_source", 10.0), ("wolf::k_row_fft", 900.0), ("wolf::k_axis_fft", 1100.0),
             ("__amd_rocclr_copyBuffer", gib2_kib)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _counter_csv(fp, "FETCH_SIZE", fetch)
    _counter_csv(wp, "WRITE_SIZE", write)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--write-traffic", str(fp), str(wp),
                        "--plan", "0,512,64", "--traffic", str(out), "--traffic-workload", "gsm256_fresnel_c64"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    rec = json.load(open(out))
    assert rec["workload"] == "gsm256_fresnel_c64"
    assert rec["plan"] == {"fused_slab": 0, "slab_chunk": 512, "col_chunk": 64, "coop_cols": 0, "coop_lookahead": 1}
    assert rec["propagate_bytes_per_launch"] == int(1200.0 * 1024 * 2.0) + int(2000.0 * 1024)
