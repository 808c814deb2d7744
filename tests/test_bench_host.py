"""bench.py host logic (no GPU): the one-GPU contract and the traffic record."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def _counters(path, counter, kern, copy, head=1.0):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for v in kern:
            w.writerow(["mp::k_head_divrem(unsigned int const*, int)", 262144, counter, head])
            w.writerow(["void k_divrem<256>(unsigned int const*, int)", 1048576, counter, v])
        w.writerow(["__amd_rocclr_copyBuffer", 4096, counter, 10.0])          # a small upload
        w.writerow(["__amd_rocclr_copyBuffer", 131072, counter, copy])        # the 256 MiB copy


def test_traffic_record_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for s in bench.TRAFFIC_SOURCES:                 # stand-in sources for the hash
        (tmp_path / s).parent.mkdir(parents=True, exist_ok=True)
        (tmp_path / s).write_text("// " + s)
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counters(f, "FETCH_SIZE", [100.0, 102.0], 131072.0)     # the copy reads back half its bytes
    _counters(w, "WRITE_SIZE", [50.0, 50.0], 262144.0)
    bench.write_traffic(str(f), str(w), "divrem_2p16_b4096")
    rec = json.load(open(tmp_path / "profiles" / "k_divrem_2p16_b4096_traffic.json"))
    assert abs(rec["fetch_factor"] - 2.0) < 1e-12 and abs(rec["write_factor"] - 1.0) < 1e-12
    # head (1 KiB each way) plus the per-instance kernel, per launch
    assert abs(rec["traffic_bytes_per_dispatch"] - 1024 * ((101.0 + 1.0) * 2 + 51.0)) < 1e-6
    assert bench.measured_traffic("divrem_2p16_b4096") == rec["traffic_bytes_per_dispatch"]
    (tmp_path / bench.TRAFFIC_SOURCES[0]).write_text("// changed")
    assert bench.measured_traffic("divrem_2p16_b4096") is None     # stale once a source changes


def test_roofline_fractions():
    """frac is the method's exact-size work at the int8 matrix peak; the
    clipped-work and vector-ALU fractions use their own counts and peak."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench.roofline(W=2e9, W_clipped=1e9, ms=1.0, kernel="k", traffic=None, algo_bytes=1)
    ops = 32 * 2e9 / 1e-3
    assert abs(r["achieved"] - ops / 1e12) < 1e-9 and r["unit"] == "int8 TOP/s"
    assert abs(r["frac"] - ops / 5.0e15) < 1e-12
    assert abs(r["frac_clipped"] - r["frac"] / 2) < 1e-12
    assert abs(r["frac_valu_peak"] - 2e12 / bench.PEAK_LIMB_PRODUCTS) < 1e-12
    assert r["peak"] == 5000.0
