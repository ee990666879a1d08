"""The counter summarizer of bench.py (--stage-table) on small synthetic
rocprofv3-shaped files: calibration on the copy dispatch, grouping by launch
shape, bandwidth and matrix-core rate arithmetic.  No GPU needed."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERNEL = "void mrinv::freq_gemm_mfma_kernel<double, 16, false, false, false>(mrinv::GemmArgs<double>)"
COPY = "__amd_rocclr_copyBuffer"

TRACE_COLS = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols, quoting=csv.QUOTE_NONNUMERIC)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_stage_table_arithmetic(tmp_path, capsys):
    # Two launches of one shape, 10 us and 30 us (mean 20 us).
    trace = [
        {"Kind": "KERNEL_DISPATCH", "Kernel_Name": COPY, "Start_Timestamp": 0, "End_Timestamp": 1000,
         "Grid_Size_X": 512, "Grid_Size_Y": 1, "Grid_Size_Z": 1},
        {"Kind": "KERNEL_DISPATCH", "Kernel_Name": KERNEL, "Start_Timestamp": 2000, "End_Timestamp": 12000,
         "Grid_Size_X": 4096, "Grid_Size_Y": 1, "Grid_Size_Z": 1},
        {"Kind": "KERNEL_DISPATCH", "Kernel_Name": KERNEL, "Start_Timestamp": 20000, "End_Timestamp": 50000,
         "Grid_Size_X": 4096, "Grid_Size_Y": 1, "Grid_Size_Z": 1},
    ]
    # The copy reads 1 GiB with FETCH_SIZE counting half of it and writes
    # 1 GiB with WRITE_SIZE exact, as measured on the device: scales 2 and 1.
    gib_kib = float(1 << 20)

    def pmc(counter, copy_kib, kern_kib):
        return [{"Dispatch_Id": 1, "Kernel_Name": COPY, "Grid_Size": 512, "Counter_Name": counter,
                 "Counter_Value": copy_kib}] + [
            {"Dispatch_Id": i, "Kernel_Name": KERNEL, "Grid_Size": 4096, "Counter_Name": counter,
             "Counter_Value": kern_kib} for i in (2, 3)]

    # Per launch: 50 MB fetched (25 MB counted), 30 MB written.
    fetch = pmc("FETCH_SIZE", gib_kib / 2, 25e6 / 1024)
    write = pmc("WRITE_SIZE", gib_kib, 30e6 / 1024)
    # MFMA: 40% busy; 2e6 MOPS x 512 flops = 1.024 GFLOP per launch.
    mfma = [{"Dispatch_Id": i, "Kernel_Name": KERNEL, "Grid_Size": 4096, "Counter_Name": n, "Counter_Value": v}
            for i in (2, 3) for n, v in (("MfmaUtil", 40.0), ("SQ_INSTS_VALU_MFMA_MOPS_F64", 2e6))]
    paths = [str(tmp_path / n) for n in ("trace.csv", "fetch.csv", "write.csv", "mfma.csv")]
    _write(paths[0], TRACE_COLS, trace)
    _write(paths[1], PMC_COLS, fetch)
    _write(paths[2], PMC_COLS, write)
    _write(paths[3], PMC_COLS, mfma)

    bench.stage_table(*paths)
    out = capsys.readouterr().out
    row = [ln for ln in out.splitlines() if "freq_gemm_mfma_kernel<double, 16, false, false, false>" in ln]
    assert len(row) == 1, out
    cells = [c.strip() for c in row[0].strip("|").split("|")]
    # kernel, grid, dispatches, avg us, share, FETCH MB, WRITE MB, GB/s, frac, busy, TFLOP/s
    assert cells[1] == "4096" and cells[2] == "2"
    assert float(cells[3]) == 20.0
    assert float(cells[4]) == 1.0                       # the copy is not part of the path
    assert abs(float(cells[5]) - 50.0) < 1e-6 and abs(float(cells[6]) - 30.0) < 1e-6
    assert abs(float(cells[7]) - 80e6 / 20e-6 / 1e9) < 0.5          # 4000 GB/s
    assert abs(float(cells[8]) - 0.5) < 1e-3
    assert float(cells[9]) == 40.0
    assert abs(float(cells[10]) - 1.024e9 / 20e-6 / 1e12) < 0.01    # 51.2 TFLOP/s


def test_write_traffic_scaling_and_hash(tmp_path, monkeypatch):
    """--traffic: scaled FETCH/WRITE bytes per launch of one kernel, keyed to
    the hash of the kernel's source; the bench line accepts the file only
    while that hash matches."""
    import argparse
    import json

    name = "freq_gemm_mfma_kernel<double, 16, false, false, false>"
    gib_kib = float(1 << 20)

    def pmc(counter, copy_kib, kern_kib):
        return [{"Dispatch_Id": 1, "Kernel_Name": COPY, "Grid_Size": 512, "Counter_Name": counter,
                 "Counter_Value": copy_kib}] + [
            {"Dispatch_Id": i, "Kernel_Name": KERNEL, "Grid_Size": 4096, "Counter_Name": counter,
             "Counter_Value": v} for i, v in ((2, kern_kib), (3, 3 * kern_kib))]

    fpath, wpath = str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv")
    _write(fpath, PMC_COLS, pmc("FETCH_SIZE", gib_kib / 2, 10e6 / 1024))   # 10 and 30 MB counted
    _write(wpath, PMC_COLS, pmc("WRITE_SIZE", gib_kib, 5e6 / 1024))        # 5 and 15 MB
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.write_traffic(argparse.Namespace(config="c2"), name, fpath, wpath)
    out = json.load(open(tmp_path / "profiles" / "traffic_c2_fp64.json"))
    assert out["dispatches"] == 2
    assert abs(out["fetch_scale"] - 2.0) < 1e-12 and abs(out["write_scale"] - 1.0) < 1e-12
    assert abs(out["fetch_bytes_per_launch"] - 40e6) < 1 and abs(out["write_bytes_per_launch"] - 10e6) < 1
    assert abs(out["bytes_per_launch"] - 50e6) < 1
    assert out["source_hash"] == bench.kernel_source_hash(name)
    assert bench.kernel_source_hash(name) != bench.kernel_source_hash("fft_pass_kernel<double, 8, 16, 0>")
