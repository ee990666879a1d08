"""Per-class tuning tables (mrinv_set_tuning_table) through the C-ABI: every
call takes its class's tuning, results stay the oracle's, batched calls with
a table agree with single calls, bad tables are refused, and the committed
table written by the autotuning script loads and covers every class."""
import json
import os

import numpy as np
import pytest
import torch

import smk_inputs as si
from tolerances import FP64_TOL, MIXED_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


TABLE = [
    {"d_lo": 1, "d_hi": 8, "n_lo": 1, "n_hi": 1 << 21, "precision": -1, "tune": {"seed_m0": 16, "lanes_fp64": 8}},
    {"d_lo": 9, "d_hi": 24, "n_lo": 1, "n_hi": 4096, "precision": "fp64", "tune": {"direct_m": 0, "lgp_max": 7}},
    {"d_lo": 9, "d_hi": 64, "n_lo": 1, "n_hi": 1 << 21, "precision": -1, "tune": {"mfma": 2, "pair_forward": 0}},
]


def test_table_tunings_keep_the_oracle_results(mr, orc):
    cases = [(5, 700, "fp64"), (5, 700, "mixed"), (16, 3000, "fp64"), (16, 3000, "bf16x3"), (33, 500, "fp64")]
    try:
        mr.set_tuning_table(TABLE)
        for d, n, prec in cases:
            q = si.weibull_kernel(d, n, 900 + d).q
            got = _np(mr.psi_inverse(q.cuda(), prec, check=True))
            tol = FP64_TOL if prec == "fp64" else MIXED_TOL
            assert float(np.max(np.abs(got - orc.psi(q.numpy())))) <= tol, (d, n, prec)
        # batched with the table: per-problem seeds and direct limits from the table
        specs = [(3, 100), (7, 2000), (12, 1000), (20, 4096), (40, 300)]
        qs = [si.weibull_kernel(d, n, 950 + i).q.cuda() for i, (d, n) in enumerate(specs)]
        outs = mr.psi_inverse_batched(qs, "fp64")
        for q, o in zip(qs, outs):
            single = mr.psi_inverse(q, "fp64")
            assert float((o - single).abs().max()) <= 1e-13
    finally:
        mr.set_tuning_table([])
    mr.sync_status()


def test_bad_tables_are_refused(mr):
    for bad in ({"d_lo": 0, "d_hi": 4, "n_lo": 1, "n_hi": 9, "precision": -1, "tune": {}},
                {"d_lo": 5, "d_hi": 4, "n_lo": 1, "n_hi": 9, "precision": -1, "tune": {}},
                {"d_lo": 1, "d_hi": 4, "n_lo": 1, "n_hi": 9, "precision": -1, "tune": {"lgp_max": 3}}):
        with pytest.raises(mr.MrinvError):
            mr.set_tuning_table([bad])
    with pytest.raises(mr.MrinvError):
        mr.set_tuning_table([{"d_lo": 1, "d_hi": 4, "n_lo": 1, "n_hi": 9, "precision": -1, "tune": {"nope": 1}}])


def test_committed_table_loads_and_covers_every_class(mr, orc):
    if not os.path.exists(mr.TUNING_TABLE):
        pytest.skip("no tuning table has been written yet")
    data = json.load(open(mr.TUNING_TABLE))
    precs = {e["precision"] for e in data["entries"]}
    for prec in precs:
        for d in (1, 8, 9, 16, 17, 33, 48, 64):
            for n in (1, 4096, 4097, 65536, 65537, 1 << 21):
                hits = [e for e in data["entries"] if e["precision"] == prec and e["d_lo"] <= d <= e["d_hi"]
                        and e["n_lo"] <= n <= e["n_hi"]]
                assert len(hits) == 1, (prec, d, n)
    try:
        assert mr.load_tuning_table() == len(data["entries"])
        q = si.lognormal_kernel(24, 5000, 960).q
        got = _np(mr.psi_inverse(q.cuda(), "fp64", check=True))
        assert float(np.max(np.abs(got[:1024] - orc.psi(q[:1024].numpy())))) <= FP64_TOL
    finally:
        mr.set_tuning_table([])
