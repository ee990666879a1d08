"""Write the per-class tuning table (tuning_table.json next to this file).

For every class of matrix dimension, horizon and precision the library's
autotuner (mrinv_autotune: a coordinate search over the fields of
mrinv_tuning_t, each candidate timed with HIP events) runs on one
representative problem, a dense semi-Markov kernel with Dirichlet jump rows
and discrete Weibull sojourns at the class's largest d and a horizon inside
the class; the chosen tuning becomes the class's entry.  Load the table with
paper_2605_30379_amd.load_tuning_table().  Needs a GPU:

    python -m paper_2605_30379_amd.tune_table [--out PATH] [--precisions fp64,mixed,bf16x3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

D_CLASSES = [(1, 8), (9, 16), (17, 32), (33, 48), (49, 64)]
N_CLASSES = [(1, 4096), (4097, 16384), (16385, 65536), (65537, 1 << 21)]


def representative_n(d_hi: int, n_lo: int, n_hi: int) -> int:
    """A horizon inside the class, kept to a size the search finishes quickly."""
    cap = 1 << 17 if d_hi <= 32 else 1 << 16
    return min(n_hi, max(n_lo, cap))


def kernel(d: int, n: int, seed: int, device):
    """q(k)_ij = p_ij f_ij(k): Dirichlet(1) rows off the diagonal, discrete
    Weibull sojourns (shape in [0.5, 2], scale in [2, 20]) renormalised on
    1..n-1, q(0) = 0."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    e = -torch.log(torch.rand(d, d, generator=g, dtype=torch.float64))
    e.fill_diagonal_(0.0)
    p = e / e.sum(dim=1, keepdim=True) if d > 1 else torch.ones(1, 1, dtype=torch.float64)
    shape = 0.5 + 1.5 * torch.rand(d, d, generator=g, dtype=torch.float64)
    scale = 2.0 + 18.0 * torch.rand(d, d, generator=g, dtype=torch.float64)
    k = torch.arange(n, dtype=torch.float64)[:, None, None]
    surv = lambda t: torch.exp(-(t.clamp(min=0) / scale) ** shape)
    f = surv(k - 1) - surv(k)
    f[0] = 0.0
    f = f / f[1:].sum(dim=0, keepdim=True).clamp(min=1e-300) if n > 1 else f
    return (p * f).to(device).contiguous()


def main():
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2605_30379_amd as mr
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=mr.TUNING_TABLE)
    ap.add_argument("--precisions", default="fp64,mixed,bf16x3")
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    base = mr.get_tuning(dev)
    entries = []
    t0 = time.time()
    for prec in args.precisions.split(","):
        for d_lo, d_hi in D_CLASSES:
            for n_lo, n_hi in N_CLASSES:
                n = representative_n(d_hi, n_lo, n_hi)
                q = kernel(d_hi, n, 1000 * d_hi + int(math.log2(n)), dev)
                mr.set_tuning(dev, **base)
                t = time.time()
                chosen = mr.autotune(q, prec)
                mr.sync_status(dev)
                diff = {k: v for k, v in chosen.items() if v != base[k]}
                print(f"[tune] {prec} d={d_hi} n={n}: {time.time() - t:.1f} s, changed {diff}", flush=True)
                entries.append({"d_lo": d_lo, "d_hi": d_hi, "n_lo": n_lo, "n_hi": n_hi, "precision": prec,
                                "tune": chosen, "representative": {"d": d_hi, "n": n}})
                del q
    mr.set_tuning(dev, **base)
    out = {"generator": "paper_2605_30379_amd/tune_table.py (mrinv_autotune per class)",
           "device": torch.cuda.get_device_name(0), "seconds": round(time.time() - t0, 1), "entries": entries}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[tune] wrote {len(entries)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
