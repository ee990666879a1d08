#!/usr/bin/env python3
"""Benchmark of psi = (e0 - q)^-1 on one MI355X: seconds per inversion and
effective TFLOP/s, FP64 and mixed precision, with a per-kernel roofline and
the CPU oracle timed beside it.

One step = one psi inversion of the workload's kernel (Gauss-Jordan seed,
every Newton doubling step and, for the mixed form, the FP64 residual sweep),
inputs already resident in HBM.  Prints ONE JSON line.

Workloads (synthetic, seeded):
  c3 (default)  d = 64, n = 262144, discrete lognormal sojourns: FP64 (value)
                and the mixed form timed beside it.
  c2            d = 16, n = 65536, Weibull sojourns, FP64 (value) and mixed.
  c1            d = 4,  n = 256, Weibull, FP64 (latency bound).
  c4            512 uneven problems in one batched call (mixed value, FP64 beside).
  c5            gradient of availability + first-entrance loss, d = 32, n = 65536.

Forms: fp64 (the value), mixed (float32 Newton + float64 residual sweeps) and
bf16x3 (the same with split-BF16 products on the matrix cores), all timed.
Accuracy (every form) is the max-abs error against the CPU oracle of psi, P,
reliability, availability and the first entrance into {d-1}, each on a prefix
of the horizon (an exact sub-problem by finite-horizon exactness).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    "c1": dict(d=4, n=256, family="weibull", seed=0, form="fp64"),
    "c2": dict(d=16, n=65536, family="weibull", seed=1, form="fp64"),
    "c3": dict(d=64, n=262144, family="lognormal", seed=3, form="fp64"),
    "c4": dict(d=0, n=0, family="mixed", seed=4, form="mixed"),
    "c5": dict(d=32, n=65536, family="weibull", seed=5, form="fp64"),
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def newton_lengths(n: int):
    """FFT lengths of the Newton steps m -> min(2m, n)."""
    out, m = [], 1
    while m < n:
        m2 = min(2 * m, n)
        out.append(1 << max(1, math.ceil(math.log2(m2))))
        m = m2
    return out


def f_nom(d: int, n: int) -> float:
    """Nominal flops of one inversion: per Newton step 5 real FFTs of
    2.5 L log2 L flops per lane on d^2 lanes, and 2 complex d x d products
    (8 d^3 flops) at each of L/2 + 1 frequencies."""
    tot = 0.0
    for L in newton_lengths(n):
        tot += 5 * d * d * 2.5 * L * math.log2(L) + 2 * (L // 2 + 1) * 8 * d ** 3
    return tot


def model_bytes(d: int, n: int, w: int) -> float:
    """Ideal traffic of one inversion: 14 L d^2 w bytes per Newton step (each
    transform a single HBM round trip, spectra of L/2+1 complex values)."""
    return sum(14.0 * L * d * d * w for L in newton_lengths(n))


CSRC = os.path.join(ROOT, "paper_2605_30379_amd", "csrc")


def source_hash(files=None) -> str:
    """Hash of the HIP sources (all of them, or the named files)."""
    h = hashlib.sha256()
    names = files if files is not None else [f for f in os.listdir(CSRC) if f.endswith((".hip", ".h"))]
    for f in sorted(names):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def kernel_source_hash(kernel: str) -> str:
    """Hash of what determines one kernel's memory traffic: the file that
    defines it and the shared headers (host-side driver code is not part)."""
    if kernel.startswith(("fft_pass", "gen_outer")):
        f = "fft.hip"
    elif kernel.startswith(("freq_", "conv_direct")):
        f = "gemm.hip"
    else:
        f = "aux.hip"
    return source_hash([f, "common.h", "kernels.h"])


def kernel_stats(mr, torch, dev):
    import ctypes

    class Stat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 96), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                    ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]

    L = mr.lib()
    L.mrinv_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mrinv_set_timing.restype = ctypes.c_int
    L.mrinv_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stat), ctypes.c_int]
    L.mrinv_kernel_stats.restype = ctypes.c_int
    h = mr._handle(dev)

    def enable(on: bool):
        L.mrinv_set_timing(h, 1 if on else 0)

    def collect():
        buf = (Stat * 256)()
        k = L.mrinv_kernel_stats(h, buf, 256)
        return [dict(name=buf[i].name.decode(), launches=int(buf[i].launches), total_ms=buf[i].total_ms,
                     bytes=buf[i].bytes, flops=buf[i].flops) for i in range(max(0, min(k, 256)))]
    return enable, collect


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def roofline_of(stats, traffic_file=None):
    """Dominant kernel by total time; algorithmic bytes / average duration."""
    if not stats:
        return None, []
    stats = sorted(stats, key=lambda s: -s["total_ms"])
    top = stats[0]
    avg_s = top["total_ms"] / top["launches"] / 1e3
    bytes_per = top["bytes"] / top["launches"]
    flops_per = top["flops"] / top["launches"]
    dbl = "double" in top["name"]
    peak_f = FP64_PEAK_TFLOPS if dbl else FP32_PEAK_TFLOPS
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    if flops_per > 0 and flops_per / max(bytes_per, 1.0) > ridge:
        achieved = flops_per / avg_s / 1e12
        roof = {"bound": "mfma" if "mfma" in top["name"] else "alu", "achieved": round(achieved, 3),
                "peak": peak_f, "unit": "TFLOP/s", "frac": round(achieved / peak_f, 4)}
    else:
        achieved = bytes_per / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof["kernel"] = top["name"]
    roof["launches"] = top["launches"]
    roof["avg_us"] = round(avg_s * 1e6, 2)
    roof["algorithmic_bytes_per_launch"] = bytes_per
    roof["traffic"] = None
    if traffic_file and os.path.exists(traffic_file):
        tr = json.load(open(traffic_file))
        if tr.get("kernel") == top["name"] and tr.get("source_hash") == kernel_source_hash(top["name"]):
            roof["traffic"] = tr.get("bytes_per_launch")
    breakdown = []
    for s in stats[:12]:
        a = s["total_ms"] / s["launches"] / 1e3
        row = {"kernel": s["name"], "launches": s["launches"], "total_ms": round(s["total_ms"], 4),
               "avg_us": round(a * 1e6, 2), "GBps": round(s["bytes"] / s["launches"] / a / 1e9, 1)}
        if s["flops"] > 0:
            row["TFLOPs"] = round(s["flops"] / s["launches"] / a / 1e12, 2)
        breakdown.append(row)
    return roof, breakdown


def hbm_measured(mr, torch, dev, roof):
    """Measured HBM ceilings (mrinv_hbm_probe, best of 3 event-timed launches
    over an 8 GiB buffer): a plain copy, and in-place reads and writes with the
    addressing of the first and the last 512-row FFT pass at 8, 16 and 32
    lanes per workgroup over 2^18 rows of 2048 complex doubles (the d=64,
    n=262144 spectra).  The dominant kernel's algorithmic bandwidth is set
    against the copy rate."""
    buf = torch.empty(1 << 30, dtype=torch.float64, device=dev)
    rates = {"copy": round(mr.hbm_probe(buf, "copy", reps=3), 1)}
    for pattern in ("pass_first", "pass_last"):
        for lanes in (8, 16, 32):
            rates[f"{pattern}_{lanes}"] = round(mr.hbm_probe(buf, pattern, lanes=lanes, reps=3), 1)
    del buf
    torch.cuda.empty_cache()
    out = {"unit": "GB/s", "rates": rates, "buffer_bytes": 1 << 33,
           "note": "best of 3 launches; bytes read + written over event-timed duration"}
    if roof:
        gbps = roof["algorithmic_bytes_per_launch"] / (roof["avg_us"] * 1e-6) / 1e9
        out["dominant_kernel_GBps"] = round(gbps, 1)
        out["dominant_kernel_frac_of_copy"] = round(gbps / rates["copy"], 4)
    print(f"[bench] hbm measured {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def write_traffic(args, kernel: str, fetch_csv: str, write_csv: str) -> None:
    """HBM traffic of one launch of `kernel` from rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled so that the 1 GiB
    device-to-device copy of --calibrate-copy (the largest copyBuffer
    dispatch) reads and writes exactly 1 GiB, then averaged over the kernel's
    dispatches.  The file carries the kernel source hash; bench.py ignores it
    once the kernels change."""
    import csv
    import re

    def rows(path, counter):
        return [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]

    def short(name):
        return re.sub(r"\(.*", "", re.sub(r"^void mrinv::", "", name)).strip()

    out = {"kernel": kernel, "source_hash": kernel_source_hash(kernel), "config": args.config,
           "form": CONFIGS[args.config]["form"]}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rr = rows(path, counter)
        cal = max(float(r["Counter_Value"]) for r in rr if "copyBuffer" in r["Kernel_Name"])
        scale = float(1 << 30) / (cal * 1024.0)
        vals = [float(r["Counter_Value"]) * 1024.0 * scale for r in rr if short(r["Kernel_Name"]) == kernel]
        if not vals:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        key = counter.split("_")[0].lower()
        out[f"{key}_scale"] = scale
        out[f"{key}_bytes_per_launch"] = sum(vals) / len(vals)
        out["dispatches"] = len(vals)
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    path = os.path.join(ROOT, "profiles", f"traffic_{args.config}_{out['form']}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))



def stage_table(trace_csv: str, fetch_csv: str, write_csv: str, mfma_csv: str) -> None:
    """Per-stage counter evidence from four rocprofv3 runs of one bench
    command: a kernel trace (durations), FETCH_SIZE, WRITE_SIZE, and MfmaUtil
    with SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32.  Dispatches are grouped by kernel,
    grid size and position in a run of adjacent dispatches of that same shape
    (the passes of one transform can share a kernel and a grid while reading
    different windows, so each pass keeps a row of its own), and then by the
    dispatch's FETCH bytes to a quarter octave (a kernel whose grid is the
    number of resident workgroups has the same grid at every transform
    length).  One command dispatches the same sequence in every profiler run,
    so the i-th dispatch of a shape is the same launch in all four files.  For
    each group it prints the
    mean duration, the scaled HBM bytes (FETCH and WRITE calibrated on the
    1 GiB copy of --calibrate-copy, as for --traffic), the achieved HBM
    bandwidth and its fraction of the 8 TB/s peak, the MFMA busy percentage
    and the matrix-core flop rate (MOPS x 512 flops).  Prints markdown."""
    import collections
    import csv
    import math
    import re

    def short(name):
        return re.sub(r"\(.*", "", re.sub(r"^void mrinv::", "", name)).strip()

    def keep(name):
        return "copyBuffer" not in name and "mrinv" in name

    def run_keys(shapes):
        """(kernel, grid, position in the run of adjacent equal shapes) for
        each dispatch of a list in dispatch order."""
        keys, prev, pos = [], None, 0
        for sh in shapes:
            pos = pos + 1 if sh == prev else 0
            keys.append((sh[0], sh[1], pos))
            prev = sh
        return keys

    def counter_keys(path):
        """Rows of a counter file and the shape key of each dispatch id, with
        the dispatch's index among the dispatches of its key."""
        rows = list(csv.DictReader(open(path)))
        first = {}
        for r in rows:
            first.setdefault(int(r["Dispatch_Id"]), r)
        ids = sorted(first)
        keys = run_keys([(short(first[i]["Kernel_Name"]), int(first[i]["Grid_Size"])) for i in ids])
        seen = collections.Counter()
        key = {}
        for i, k in zip(ids, keys):
            key[i] = (k, seen[k])
            seen[k] += 1
        return rows, key

    # Size class of each dispatch: log2 of its FETCH counter to a quarter
    # octave, by shape key and index.
    frows, fkey = counter_keys(fetch_csv)
    fclass = {}
    for r in frows:
        if r["Counter_Name"] == "FETCH_SIZE":
            v = float(r["Counter_Value"])
            fclass[fkey[int(r["Dispatch_Id"])]] = round(4 * math.log2(v)) if v > 0 else -1

    def group(k, idx):
        return k + (fclass.get((k, idx), -1),)

    dur = collections.defaultdict(list)
    trace = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    shapes = [(short(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
              for r in trace]
    seen = collections.Counter()
    for r, k in zip(trace, run_keys(shapes)):
        if keep(r["Kernel_Name"]):
            dur[group(k, seen[k])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
        seen[k] += 1

    def counters(path, names):
        out = collections.defaultdict(lambda: collections.defaultdict(list))
        rows, key = counter_keys(path)
        for r in rows:
            if r["Counter_Name"] in names and keep(r["Kernel_Name"]):
                k, idx = key[int(r["Dispatch_Id"])]
                out[group(k, idx)][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return rows, out

    scaled = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows, c = counters(path, {counter})
        cal = max(float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"])
        scale = float(1 << 30) / (cal * 1024.0)
        for k, v in c.items():
            vals = v[counter]
            scaled.setdefault(k, {})[counter] = sum(vals) / len(vals) * 1024.0 * scale
    _, mf = counters(mfma_csv, {"MfmaUtil", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32"})

    def mean(xs):
        return sum(xs) / len(xs) if xs else 0.0

    total = sum(sum(v) for v in dur.values())
    print("| kernel | grid | run pos | dispatches | avg us | share of kernel time | FETCH MB | WRITE MB | HBM GB/s | of 8 TB/s "
          "| MFMA busy % | MFMA TFLOP/s |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        t = sum(dur[k]) / len(dur[k])
        share = sum(dur[k]) / total
        if share < 0.01:
            continue
        f = scaled.get(k, {}).get("FETCH_SIZE")
        w = scaled.get(k, {}).get("WRITE_SIZE")
        bw = (f + w) / t / 1e9 if f is not None and w is not None else None
        m = mf.get(k, {})
        util = mean(m["MfmaUtil"]) if m.get("MfmaUtil") else None
        mops = mean(m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [])) + mean(m.get("SQ_INSTS_VALU_MFMA_MOPS_F32", []))
        tf = mops * 512 / t / 1e12 if mops > 0 else None

        def fmt(x, spec):
            return "—" if x is None else format(x, spec)
        print(f"| `{k[0]}` | {k[1]} | {k[2]} | {len(dur[k])} | {t * 1e6:.2f} | {share:.3f} | {fmt(f and f / 1e6, '.2f')} "
              f"| {fmt(w and w / 1e6, '.2f')} | {fmt(bw, '.0f')} | {fmt(bw and bw / 8000.0, '.3f')} "
              f"| {fmt(util, '.1f')} | {fmt(tf, '.2f')} |")
    print(f"\nKernel time over the trace: {total * 1e3:.3f} ms in {sum(len(v) for v in dur.values())} dispatches; "
          "groups under 1% of it are not listed.")

def cpu_baseline(cfg, budget_s: float):
    """The oracle's left recursion on a prefix n' of the same kernel (finite-
    horizon exactness makes the prefix a valid sub-problem), sized to about
    budget_s seconds; the full-horizon time is extrapolated by its quadratic
    cost (n / n')^2."""
    import oracle
    import smk_inputs as si
    d, n = cfg["d"], cfg["n"]
    gen = si.family_kernel

    def run(npre):
        q = gen(cfg["family"], d, n, cfg["seed"], n_rows=npre).q.numpy()
        t = time.perf_counter()
        oracle.psi(q)
        return time.perf_counter() - t

    npre = min(n, 256)
    t = run(npre)
    while npre < n and t < budget_s / 4:
        nxt = min(n, npre * 2)
        pred = t * (nxt / npre) ** 2
        if pred > budget_s * 1.5:
            break
        npre = nxt
        t = run(npre)
    t_full = t * (n / npre) ** 2
    return {"value": f_nom(d, n) / t_full / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"left coefficient recursion on the first {npre} of {n} coefficients (d={d}), "
                      f"{t:.2f} s measured, full horizon {t_full:.1f} s extrapolated by (n/n')^2",
            "sample_seconds": round(t, 3), "extrapolated_full_seconds": round(t_full, 2)}


PREFIX = {  # oracle prefixes per config: psi and P, then reliability, availability, first entrance
    "c1": (256, 256), "c2": (2048, 8192), "c3": (1024, 4096), "c5": (2048, 8192),
}


def accuracy(cfg, q, forms, mr, torch, si, dev):
    """Max-abs errors against the oracle of psi, P = psi*Hbar, reliability
    (up set = first d/2 states, alpha = e0), availability (same up set) and
    the first entrance into {d-1} (alpha = e0), per form, on prefixes."""
    import numpy as np

    import oracle
    d, n = cfg["d"], cfg["n"]
    n_psi, n_fun = (min(n, v) for v in PREFIX.get(cfg.get("name", ""), (1024, 4096)))
    qh = q[:n_fun].cpu().numpy()
    up = np.array([1] * (d // 2) + [0] * (d - d // 2), dtype=np.int32)
    alpha = np.eye(d)[0]
    inD = np.zeros(d, dtype=np.int32)
    inD[d - 1] = 1
    t0 = time.perf_counter()
    ref_psi = oracle.psi(qh[:n_psi])
    ref = {"psi": ref_psi, "P": oracle.transition(ref_psi, qh[:n_psi]),
           "reliability": oracle.reliability(qh, up, alpha), "availability": oracle.availability(qh, up, alpha),
           "first_entrance": oracle.first_entrance(qh, inD, alpha)[1]}
    acc = {"oracle_prefix": {"psi": n_psi, "P": n_psi, "reliability": n_fun, "availability": n_fun,
                             "first_entrance": n_fun},
           "oracle_seconds": round(time.perf_counter() - t0, 2)}
    got = {}
    for form in forms:
        psi = mr.psi_inverse(q, form, check=True)
        P = mr.transition(psi, q)
        A = mr.availability(P, up, alpha)
        rows = float((P.sum(dim=2) - 1).abs().max())
        Pp = P[:n_psi].cpu().numpy()
        del P
        R = mr.reliability(q, up, alpha, precision=form)
        F = mr.first_entrance(q, inD, alpha, precision=form)[1]
        e = {"psi": float(np.max(np.abs(psi[:n_psi].cpu().numpy() - ref["psi"]))),
             "P": float(np.max(np.abs(Pp - ref["P"]))),
             "reliability": float(np.max(np.abs(R[:n_fun].cpu().numpy() - ref["reliability"]))),
             "availability": float(np.max(np.abs(A[:n_fun].cpu().numpy() - ref["availability"]))),
             "first_entrance": float(np.max(np.abs(F[:n_fun].cpu().numpy() - ref["first_entrance"]))),
             "P_row_sums_minus_1_whole_horizon": rows}
        acc[form] = e
        got[form] = psi
    if "fp64" in got and "mixed" in got:
        acc["mixed_vs_fp64_psi_whole_horizon"] = float((got["mixed"] - got["fp64"]).abs().max())
    del got
    gk = si.geometric_kernel(d, n, 2, device=dev)
    ks = np.unique(np.linspace(0, n - 1, 24).astype(int))
    gref = oracle.geometric_psi(gk.params["M"], gk.params["a"], ks)
    kt = torch.as_tensor(ks, device=dev)
    for form in forms:
        acc[form]["psi_markov_closed_form_whole_horizon"] = float(
            np.max(np.abs(mr.psi_inverse(gk.q, form)[kt].cpu().numpy() - gref)))
    mr.sync_status(dev)
    return acc


def run_batched(args, mr, torch, si, dev):
    """512 uneven problems (d in 3..48, n log-uniform in [1024, 32768]) in one
    batched call per step; every form timed, also as one call per problem.
    The value is the mixed form's effective TFLOP/s; the FP64 form is measured
    against its byte model (sum over problems of 14 L d^2 w per Newton step)
    and the dominant kernel's roofline comes from the library's launch timer."""
    work = si.batch_workload(CONFIGS["c4"]["seed"], 512)
    n_table = 0 if args.no_tuning_table else mr.load_tuning_table(device=dev)
    print(f"[bench] c4: tuning table with {n_table} entries", file=sys.stderr, flush=True)
    qs = [si.family_kernel(w["family"], w["d"], w["n"], w["seed"], device=dev).q for w in work]
    torch.cuda.synchronize()
    fl = sum(f_nom(w["d"], w["n"]) for w in work)
    mb64 = sum(model_bytes(w["d"], w["n"], 8) for w in work)
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for form in forms:
        plan = mr.BatchedPlan(qs, form)
        ms = time_steps(plan.launch, args.steps, args.warmup, torch)
        mr.sync_status(dev)
        ms_single = time_steps(lambda: [mr.psi_inverse(q, form) for q in qs], max(1, args.steps // 4), 1, torch)
        res[form] = {"ms": ms, "tflops": fl / (ms * 1e-3) / 1e12, "ms_one_call_each": ms_single}
        print(f"[bench] c4 {form}: batched {ms:.3f} ms, one call each {ms_single:.3f} ms", file=sys.stderr, flush=True)
        del plan
    value_form = "mixed" if "mixed" in res else forms[0]
    roof = breakdown = None
    if "fp64" in res:
        plan = mr.BatchedPlan(qs, "fp64")
        enable, collect = kernel_stats(mr, torch, dev)
        enable(True)
        plan.launch()
        stats = collect()
        enable(False)
        roof, breakdown = roofline_of(stats, os.path.join(ROOT, "profiles", "traffic_c4_fp64.json"))
        del plan
    v = res[value_form]
    line = {
        "metric": "psi inversion sec & effective TFLOP/s, mixed vs FP64 on 1 GPU @ max err<=1e-10",
        "value": round(v["tflops"], 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(v["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "c4: 512 uneven problems, d in 3..48, n log-uniform in [1024, 32768], "
                               "Weibull or lognormal, one batched launch sequence per step (prepared plan)",
                   "problems": 512, "form": value_form},
        "forms": {f: {k: round(x, 4) for k, x in r.items()} for f, r in res.items()},
        "speedup_vs_fp64": ({f: round(res["fp64"]["ms"] / res[f]["ms"], 3) for f in res} if "fp64" in res else None),
        "model_bytes_fp64": mb64,
        "path_roofline_frac_fp64": (round(mb64 / (HBM_PEAK_GBS * 1e9) / (res["fp64"]["ms"] * 1e-3), 4)
                                    if "fp64" in res else None),
        "roofline_fp64": roof, "kernels_fp64": breakdown,
        "nominal_flops": fl, "tuning_table_entries": n_table, "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)


def run_gradient(args, mr, torch, si, dev):
    """Loss = sum_k A(k) + F_{d-1}(n-1) and its gradient with respect to all
    Weibull shapes, scales and logits (d = 32, n = 65536), one step = forward
    plus backward through the adjoint kernels."""
    d, n = 32, 65536
    shape, scale, logits = si.weibull_params(d, CONFIGS["c5"]["seed"], device=dev)
    up = torch.tensor([1.0] * 16 + [0.0] * 16, dtype=torch.float64)
    alpha = torch.zeros(d, dtype=torch.float64)
    alpha[0] = 1.0
    C = list(range(d - 1))
    aC = torch.zeros(d - 1, dtype=torch.float64)
    aC[0] = 1.0

    def step():
        ps = [t.clone().requires_grad_(True) for t in (shape, scale, logits)]
        q = si.weibull_kernel_from_params(*ps, n)
        psi = mr.PsiInverse.apply(q)
        P = mr.Transition.apply(psi, q)
        A = mr.Contract.apply(P, alpha, up)
        g = mr.RenewalApply.apply(mr.PsiInverse.apply(mr.GatherBlock.apply(q, C, C)), mr.GatherBlock.apply(q, C, [d - 1]))
        F = mr.Contract.apply(g, aC, torch.ones(1, dtype=torch.float64), True)
        (A.sum() + F[-1]).backward()
        return ps

    ms = time_steps(step, args.steps, args.warmup, torch)
    q5 = si.weibull_kernel(d, n, CONFIGS["c5"]["seed"], device=dev).q
    fwd_ms = time_steps(lambda: mr.psi_inverse(q5), args.steps, 1, torch)
    line = {
        "metric": "psi inversion sec & effective TFLOP/s, mixed vs FP64 on 1 GPU @ max err<=1e-10",
        "value": round(2 * f_nom(d, n) / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c5: gradient of sum_k A(k) + F_{d-1}(n-1), d=32, n=65536, Weibull, "
                               "2976 live parameters, forward + backward", "d": d, "n": n},
        "psi_inverse_ms": round(fwd_ms, 4), "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy checks against the oracle")
    ap.add_argument("--no-tuning-table", action="store_true", help="c4: do not load the per-class tuning table")
    ap.add_argument("--no-hbm-probe", action="store_true", help="skip the measured HBM ceilings")
    ap.add_argument("--forms", default="fp64,mixed,bf16x3", help="comma-separated forms to time (value form first)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM counter runs)")
    ap.add_argument("--stage-table", nargs=4, metavar=("TRACE_CSV", "FETCH_CSV", "WRITE_CSV", "MFMA_CSV"),
                    help="print per-stage counter evidence (duration, HBM bytes and bandwidth, MFMA busy) from four "
                         "rocprofv3 runs of one --calibrate-copy bench command, then exit")
    ap.add_argument("--traffic", nargs=3, metavar=("KERNEL", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<config>_<form>.json for KERNEL from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, then WRITE_SIZE) of a --calibrate-copy bench command, then exit")
    args = ap.parse_args()

    if args.stage_table:
        return stage_table(*args.stage_table)
    if args.traffic:
        return write_traffic(args, *args.traffic)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path is single-GPU by design "
              f"and sharding is described, not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_30379_amd as mr
    import smk_inputs as si

    cfg = dict(CONFIGS[args.config], name=args.config)
    d, n = cfg["d"], cfg["n"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.config == "c4":
        return run_batched(args, mr, torch, si, dev)
    if args.config == "c5":
        return run_gradient(args, mr, torch, si, dev)
    print(f"[bench] config {args.config}: d={d} n={n} {cfg['family']}", file=sys.stderr, flush=True)
    q = si.family_kernel(cfg["family"], d, n, cfg["seed"], device=dev).q
    torch.cuda.synchronize()
    if args.calibrate_copy:
        # A plain copy of known size: 1 GiB read + 1 GiB written.
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    forms = [f for f in args.forms.split(",") if f]
    if cfg["form"] not in forms:
        forms.insert(0, cfg["form"])
    res = {}
    for form in forms:
        ms = time_steps(lambda: mr.psi_inverse(q, form), args.steps, args.warmup, torch)
        mr.sync_status(dev)
        res[form] = {"ms": ms, "tflops": f_nom(d, n) / (ms * 1e-3) / 1e12}
        print(f"[bench] {form}: {ms:.4f} ms/inversion, {res[form]['tflops']:.3f} effective TFLOP/s",
              file=sys.stderr, flush=True)

    # Per-kernel timing of the value form (separate run; the library stamps each
    # launch with dispatch-packet events).
    value_form = cfg["form"]
    enable, collect = kernel_stats(mr, torch, dev)
    enable(True)
    for _ in range(max(1, min(args.steps, 5))):
        mr.psi_inverse(q, value_form)
    stats = collect()
    enable(False)
    traffic_file = os.path.join(ROOT, "profiles", f"traffic_{args.config}_{value_form}.json")
    roof, breakdown = roofline_of(stats, traffic_file)
    path_ms = sum(s["total_ms"] for s in stats) / max(1, min(args.steps, 5))
    hbm = None if args.no_hbm_probe else hbm_measured(mr, torch, dev, roof)

    # Accuracy of both forms against the oracle (prefixes: exact sub-problems by
    # finite-horizon exactness), the mixed form against FP64 over the whole
    # horizon, and the Markov closed form at sampled coefficients.
    acc = {}
    if not args.no_check:
        acc = accuracy(cfg, q, forms, mr, torch, si, dev)
        print(f"[bench] accuracy {json.dumps(acc)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, args.cpu_budget)
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

    v = res[value_form]
    w = 8 if value_form == "fp64" else 4
    line = {
        "metric": "psi inversion sec & effective TFLOP/s, mixed vs FP64 on 1 GPU @ max err<=1e-10",
        "value": round(v["tflops"], 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(v["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if value_form == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: psi=(e0-q)^-1, d={d}, n={n}, {cfg['family']} sojourns, "
                               f"{value_form}", "d": d, "n": n, "form": value_form, "seed": cfg["seed"]},
        "seconds_per_inversion": {f: round(res[f]["ms"] / 1e3, 7) for f in forms},
        "effective_tflops": {f: round(res[f]["tflops"], 4) for f in forms},
        "mixed_speedup_vs_fp64": (round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
                                  if "fp64" in res and "mixed" in res else None),
        "speedup_vs_fp64": ({f: round(res["fp64"]["ms"] / res[f]["ms"], 3) for f in forms}
                            if "fp64" in res else None),
        "nominal_flops": f_nom(d, n),
        "model_bytes_fp64": model_bytes(d, n, 8),
        "path_roofline_frac_fp64": (round(model_bytes(d, n, 8) / (HBM_PEAK_GBS * 1e9) / (res["fp64"]["ms"] * 1e-3), 4)
                                    if "fp64" in res else None),
        "kernel_time_ms_per_step": round(path_ms, 4),
        "accuracy": acc,
        "roofline": roof,
        "hbm_measured": hbm,
        "kernels": breakdown,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
