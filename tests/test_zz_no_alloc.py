"""mrinv_psi_inverse_noalloc, the entry point for callers that cannot
allocate: called through the C-ABI, its output must equal that of
mrinv_psi_inverse (same kernels, same plan) on two calls in a row, the second
with a smaller input, and sizes beyond the library-owned array are refused."""
import ctypes

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


def _noalloc(mr, q, psi, prec):
    n, d, _ = q.shape
    L = mr.lib()
    h = mr._handle(q.device)
    return L.mrinv_psi_inverse_noalloc(h, ctypes.c_void_p(q.data_ptr()), d, n, mr._PREC[prec],
                                       ctypes.c_void_p(psi.data_ptr()))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_the_workspace_entry_point(mr, orc, prec):
    cases = [(8, 3000, 301), (3, 500, 302)]          # second call smaller than the first
    outs = []
    for d, n, seed in cases:
        print(f"[noalloc] {prec} d={d} n={n}", flush=True)
        q = si.weibull_kernel(d, n, seed, device="cuda").q
        ref = mr.psi_inverse(q, prec)
        got = torch.full_like(q, float("nan"))
        assert _noalloc(mr, q, got, prec) == 0, mr.lib().mrinv_last_error()
        mr.sync_status()
        outs.append((q, got.clone(), ref))
    for (q, got, ref) in outs:
        tol = FP64_TOL if prec == "fp64" else MIXED_TOL
        assert torch.equal(got, ref)                                  # same kernels, same bits
        assert float((got - ref).abs().max()) <= tol
        e = float(np.max(np.abs(got[:256].cpu().numpy() - orc.psi(q[:256].cpu().numpy()))))
        assert e <= tol


def test_noalloc_refuses_sizes_beyond_the_array(mr):
    d, n = 64, 4096                                   # about 400 MB of workspace
    need = mr.workspace_size("psi_inverse", d, n)
    assert need > mr.NOALLOC_SCRATCH_BYTES
    q = torch.zeros((n, d, d), dtype=torch.float64, device="cuda")
    psi = torch.empty_like(q)
    assert _noalloc(mr, q, psi, "fp64") == 4          # MRINV_E_WORKSPACE, nothing enqueued
    assert b"library-owned" in mr.lib().mrinv_last_error()
    with pytest.raises(mr.MrinvError):
        mr.psi_inverse_noalloc(q, psi)
    mr.sync_status()
