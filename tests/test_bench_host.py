"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte counts the roofline
divides by, and the counter-to-traffic reduction with its calibration and source digest."""
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
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_headline_step():
    # 16 images of 512 x 512, 49 real filters: x and y (4 B per pixel each), c written and read
    # (4 B per coefficient each), and the real filter sets of 257 half-spectrum columns, once per direction
    B, N, M, K = 16, 512, 512, 49
    assert (bench.B, bench.N, bench.M) == (B, N, M)
    want = B * N * M * 4 * 2 + B * K * N * M * 4 * 2 + 2 * K * N * (M // 2 + 1) * 4
    assert bench.path_algorithmic_bytes(K, True) == want == 1729302528
    per_kernel = sum(bench.kernel_algorithmic_bytes(k, K, True)
                     for k in ("rows_r2c_images", "cols_fwd", "rows_c2r_coeffs", "rows_r2c_coeffs", "cols_inv",
                               "rows_c2r_images"))
    assert per_kernel == want
    assert bench.kernel_algorithmic_bytes("rows_c2r_coeffs", K, True) == B * K * N * M * 4
    # the whole-plane forward: its plane kernel reads the filters and writes the coefficients, the
    # column-spectra pass moves none of the method's bytes; the step's total is the same
    plane = sum(bench.kernel_algorithmic_bytes(k, K, True, plane_fwd=True)
                for k in ("rows_r2c_images", "cols_fwd", "plane_fwd", "rows_r2c_coeffs", "cols_inv",
                          "rows_c2r_images"))
    assert plane == want
    assert bench.kernel_algorithmic_bytes("cols_fwd", K, True, plane_fwd=True) == 0
    assert bench.exchange_bytes("plane_fwd", K, plane_fwd=True) == B * N * (M // 2) * 8


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_calibrates_and_keys_by_source(tmp_path):
    cal = 1 << 29
    kern = "void shear::(anonymous namespace)::k_rows_c2r<512, 1, 16>(HIP_vector_type<float, 2u> const*, float*)"
    # the copy kernel's FETCH_SIZE reads half its bytes, WRITE_SIZE all of them (KiB, summed over the
    # counter's instances within a dispatch)
    _counter_csv(tmp_path / "calf.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "copy", "Counter_Name": "FETCH_SIZE", "Counter_Value": cal / 2048 / 2},
        {"Dispatch_Id": 1, "Kernel_Name": "copy", "Counter_Name": "FETCH_SIZE", "Counter_Value": cal / 2048 / 2}])
    _counter_csv(tmp_path / "calw.csv", [
        {"Dispatch_Id": 1, "Kernel_Name": "copy", "Counter_Name": "WRITE_SIZE", "Counter_Value": cal / 1024}])
    _counter_csv(tmp_path / "fetch.csv", [
        {"Dispatch_Id": 5, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
        {"Dispatch_Id": 5, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 500.0},
        {"Dispatch_Id": 9, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1700.0}])
    _counter_csv(tmp_path / "write.csv", [
        {"Dispatch_Id": 5, "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": 3000.0},
        {"Dispatch_Id": 9, "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": 3200.0}])
    # VALU instructions: plain counts summed over the counter's instances, averaged over dispatches
    _counter_csv(tmp_path / "valu.csv", [
        {"Dispatch_Id": 5, "Kernel_Name": kern, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 4.0e7},
        {"Dispatch_Id": 5, "Kernel_Name": kern, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 4.0e7},
        {"Dispatch_Id": 9, "Kernel_Name": kern, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 9.0e7}])
    src = tmp_path / "kernels.hip"
    src.write_text("// one version of the kernels\n")
    out = tmp_path / "counters.json"
    assert bench.traffic_summary(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"), str(tmp_path / "calf.csv"),
                                 str(tmp_path / "calw.csv"), cal, out_path=str(out), src=str(src),
                                 valu_csv=str(tmp_path / "valu.csv")) == 0
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    ent = rec["kernels"]["rows_c2r_coeffs"]
    assert ent["fetch_bytes"] == pytest.approx(2.0 * 1024 * (1500.0 + 1700.0) / 2)  # mean over dispatches, x 2
    assert ent["write_bytes"] == pytest.approx(1024 * (3000.0 + 3200.0) / 2)
    assert ent["valu_wave_instructions"] == pytest.approx(8.5e7)
    got = bench.traffic_from_profiles("rows_c2r_coeffs", 1.0, path=str(out), src=str(src))
    assert got == pytest.approx(ent["fetch_bytes"] + ent["write_bytes"])
    # VALU side: 8.5e7 wave instructions at 256 CUs x 2.4 GHz x 1 per clock take 0.1383 ms
    v = bench.valu_bound("rows_c2r_coeffs", 0.2766, path=str(out), src=str(src))
    assert v["min_ms"] == pytest.approx(8.5e7 / 614.4e9 * 1e3) and v["frac"] == pytest.approx(0.5, rel=1e-3)
    # counters taken on one workload say nothing about another (a 256x256 layer, say)
    assert bench.traffic_from_profiles("rows_c2r_coeffs", 1.0, path=str(out), src=str(src),
                                       workload="32x256x256x33") is None
    assert bench.valu_bound("rows_c2r_coeffs", 0.2766, path=str(out), src=str(src), workload="32x256x256x33") is None
    # ... until that workload's own counters are added beside the record (its 256-column kernels)
    k256 = "void shear::(anonymous namespace)::k_plane_fwd<256, 256>(HIP_vector_type<float, 2u> const*, float*)"
    _counter_csv(tmp_path / "fetch2.csv", [
        {"Dispatch_Id": 3, "Kernel_Name": k256, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0},
        {"Dispatch_Id": 3, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 7.0}])
    _counter_csv(tmp_path / "write2.csv", [
        {"Dispatch_Id": 3, "Kernel_Name": k256, "Counter_Name": "WRITE_SIZE", "Counter_Value": 300.0}])
    assert bench.traffic_summary(str(tmp_path / "fetch2.csv"), str(tmp_path / "write2.csv"), str(tmp_path / "calf.csv"),
                                 str(tmp_path / "calw.csv"), cal, out_path=str(out), src=str(src),
                                 workload="32x256x256x33") == 0
    got = bench.traffic_from_profiles("plane_fwd", 1.0, path=str(out), src=str(src), workload="32x256x256x33")
    assert got == pytest.approx(2.0 * 1024 * 100.0 + 1024 * 300.0)
    # the 512-column kernel is not one of this workload's kinds, and the headline record is unchanged
    assert bench.traffic_from_profiles("rows_c2r_coeffs", 1.0, path=str(out), src=str(src),
                                       workload="32x256x256x33") is None
    assert bench.traffic_from_profiles("rows_c2r_coeffs", 1.0, path=str(out), src=str(src)) == pytest.approx(
        ent["fetch_bytes"] + ent["write_bytes"])
    # a changed kernel source makes the stored counters stale
    src.write_text("// another version of the kernels\n")
    assert bench.traffic_from_profiles("rows_c2r_coeffs", 1.0, path=str(out), src=str(src)) is None
    assert bench.valu_bound("rows_c2r_coeffs", 0.2766, path=str(out), src=str(src)) is None
