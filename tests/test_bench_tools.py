"""The counter summarizer of bench.py (--stage-table) on small synthetic
rocprofv3-shaped files: calibration on the copy dispatch, grouping by launch
shape and position in a run of adjacent equal shapes, bandwidth and
matrix-core rate arithmetic.  No GPU needed."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERNEL = "void mrinv::freq_gemm_mfma_kernel<double, 16, false, false, false>(mrinv::GemmArgs<double>)"
OTHER = "void mrinv::fft_pass_kernel<double, 8, 16, 1>(mrinv::PassGeom)"
COPY = "__amd_rocclr_copyBuffer"

TRACE_COLS = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols, quoting=csv.QUOTE_NONNUMERIC)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_stage_table_arithmetic(tmp_path, capsys):
    # Dispatch order: copy, KERNEL (10 us), OTHER, KERNEL (30 us), KERNEL (5 us).
    # The first two KERNEL launches are both first in their run (mean 20 us);
    # the third directly follows a launch of its own shape and gets a row of
    # its own (run position 1), as the second pass of a transform does.
    def launch(i, name, t0, t1, grid):
        return {"Kind": "KERNEL_DISPATCH", "Dispatch_Id": i, "Kernel_Name": name, "Start_Timestamp": t0,
                "End_Timestamp": t1, "Grid_Size_X": grid, "Grid_Size_Y": 1, "Grid_Size_Z": 1}
    trace = [launch(1, COPY, 0, 1000, 512), launch(2, KERNEL, 2000, 12000, 4096),
             launch(3, OTHER, 13000, 14000, 4096), launch(4, KERNEL, 20000, 50000, 4096),
             launch(5, KERNEL, 51000, 56000, 4096)]
    # The copy reads 1 GiB with FETCH_SIZE counting half of it and writes
    # 1 GiB with WRITE_SIZE exact, as measured on the device: scales 2 and 1.
    gib_kib = float(1 << 20)

    def pmc(counter, copy_kib, kern_kib, last_kib):
        return ([{"Dispatch_Id": 1, "Kernel_Name": COPY, "Grid_Size": 512, "Counter_Name": counter,
                  "Counter_Value": copy_kib},
                 {"Dispatch_Id": 3, "Kernel_Name": OTHER, "Grid_Size": 4096, "Counter_Name": counter,
                  "Counter_Value": 1.0}] +
                [{"Dispatch_Id": i, "Kernel_Name": KERNEL, "Grid_Size": 4096, "Counter_Name": counter,
                  "Counter_Value": v} for i, v in ((2, kern_kib), (4, kern_kib), (5, last_kib))])

    # Per launch in run position 0: 50 MB fetched (25 MB counted), 30 MB
    # written; in run position 1: 10 MB fetched, 5 MB written.
    fetch = pmc("FETCH_SIZE", gib_kib / 2, 25e6 / 1024, 5e6 / 1024)
    write = pmc("WRITE_SIZE", gib_kib, 30e6 / 1024, 5e6 / 1024)
    # MFMA: 40% busy; 2e6 MOPS x 512 flops = 1.024 GFLOP per launch.
    mfma = [{"Dispatch_Id": i, "Kernel_Name": KERNEL, "Grid_Size": 4096, "Counter_Name": n, "Counter_Value": v}
            for i in (2, 4, 5) for n, v in (("MfmaUtil", 40.0), ("SQ_INSTS_VALU_MFMA_MOPS_F64", 2e6))]
    paths = [str(tmp_path / n) for n in ("trace.csv", "fetch.csv", "write.csv", "mfma.csv")]
    _write(paths[0], TRACE_COLS, trace)
    _write(paths[1], PMC_COLS, fetch)
    _write(paths[2], PMC_COLS, write)
    _write(paths[3], PMC_COLS, mfma)

    bench.stage_table(*paths)
    out = capsys.readouterr().out
    rows = [[c.strip() for c in ln.strip().strip("|").split("|")]
            for ln in out.splitlines() if "freq_gemm_mfma_kernel<double, 16, false, false, false>" in ln]
    assert len(rows) == 2, out
    by_pos = {r[2]: r for r in rows}
    # kernel, grid, run pos, dispatches, avg us, share, FETCH MB, WRITE MB, GB/s, frac, busy, TFLOP/s
    cells = by_pos["0"]
    assert cells[1] == "4096" and cells[3] == "2"
    assert float(cells[4]) == 20.0
    assert abs(float(cells[5]) - 40.0 / 46.0) < 1e-3    # the copy is not part of the path
    assert abs(float(cells[6]) - 50.0) < 1e-6 and abs(float(cells[7]) - 30.0) < 1e-6
    assert abs(float(cells[8]) - 80e6 / 20e-6 / 1e9) < 0.5          # 4000 GB/s
    assert abs(float(cells[9]) - 0.5) < 1e-3
    assert float(cells[10]) == 40.0
    assert abs(float(cells[11]) - 1.024e9 / 20e-6 / 1e12) < 0.01    # 51.2 TFLOP/s
    last = by_pos["1"]
    assert last[3] == "1" and float(last[4]) == 5.0
    assert abs(float(last[6]) - 10.0) < 1e-6 and abs(float(last[7]) - 5.0) < 1e-6


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


def test_stage_table_splits_one_shape_by_fetch_bytes(tmp_path, capsys):
    """A kernel launched with the same grid at two transform lengths (the
    resident-grid product) keeps one row per length: dispatches of one shape
    are grouped by their FETCH bytes to a quarter octave, and each row's
    duration comes from the matching dispatches of the trace run."""
    other = OTHER
    grid = 262144
    # KERNEL at 4 GB, OTHER, KERNEL at 1 GB, OTHER, KERNEL at 4.1 GB (same class as 4 GB).
    spec = [(2, KERNEL, 40.0, 4e9), (3, other, 1.0, 1e6), (4, KERNEL, 10.0, 1e9), (5, other, 1.0, 1e6),
            (6, KERNEL, 44.0, 4.1e9)]
    trace = [{"Kind": "KERNEL_DISPATCH", "Dispatch_Id": 1, "Kernel_Name": COPY, "Start_Timestamp": 0,
              "End_Timestamp": 1000, "Grid_Size_X": 512, "Grid_Size_Y": 1, "Grid_Size_Z": 1}]
    t = 2000
    for i, name, us, _ in spec:
        trace.append({"Kind": "KERNEL_DISPATCH", "Dispatch_Id": i, "Kernel_Name": name, "Start_Timestamp": t,
                      "End_Timestamp": t + int(us * 1000), "Grid_Size_X": grid, "Grid_Size_Y": 1,
                      "Grid_Size_Z": 1})
        t += int(us * 1000) + 500
    gib_kib = float(1 << 20)

    def pmc(counter, copy_kib, scale):
        return [{"Dispatch_Id": 1, "Kernel_Name": COPY, "Grid_Size": 512, "Counter_Name": counter,
                 "Counter_Value": copy_kib}] + [
            {"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
             "Counter_Value": b / scale / 1024} for i, name, _, b in spec]
    paths = [str(tmp_path / n) for n in ("trace.csv", "fetch.csv", "write.csv", "mfma.csv")]
    _write(paths[0], TRACE_COLS, trace)
    _write(paths[1], PMC_COLS, pmc("FETCH_SIZE", gib_kib / 2, 2.0))
    _write(paths[2], PMC_COLS, pmc("WRITE_SIZE", gib_kib, 2.0))
    _write(paths[3], PMC_COLS, [])
    bench.stage_table(*paths)
    out = capsys.readouterr().out
    rows = [[c.strip() for c in ln.strip().strip("|").split("|")]
            for ln in out.splitlines() if "freq_gemm_mfma_kernel<double, 16, false, false, false>" in ln]
    assert len(rows) == 2, out
    big = [r for r in rows if float(r[6]) > 3000][0]
    small = [r for r in rows if float(r[6]) < 3000][0]
    assert big[3] == "2" and abs(float(big[4]) - 42.0) < 1e-6          # mean of 40 and 44 us
    assert abs(float(big[6]) - 4050.0) < 1e-6                          # mean of 4000 and 4100 MB
    assert small[3] == "1" and abs(float(small[4]) - 10.0) < 1e-6 and abs(float(small[6]) - 1000.0) < 1e-6
