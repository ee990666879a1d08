"""Parity at the headline workload: d = 64, n = 262144 (2^18), discrete
lognormal sojourns (seed 3), FP64 and both mixed forms (float32 products and
the split-BF16 products the workload names), through the C-ABI in the launch
configuration bench.py times.

The quadratic oracle cannot form all 2^18 coefficients, so the evidence is
layered (every reference comes from the oracle, never from the GPU path):
  * the whole matrix psi(k) on the prefix k < 2048 and the alpha-row
    alpha psi(k) (alpha = e0) on k < 16384: exact sub-problems by
    finite-horizon exactness (Proposition 2.3);
  * the left residual e0 - A*psi at 16 coefficients spread over the whole
    horizon, up to k = n - 1, each by the oracle's direct sum over
    l = 0..k (Proposition 2.6 bounds the error by the residual);
  * P, reliability (up set = states 0..31), availability and the first
    entrance into {d-1} on prefixes, plus the exact row-sum identity of P at
    every k.
"""
import time

import numpy as np
import pytest
import torch

import smk_inputs as si
from tolerances import FP64_TOL, MIXED_TOL, fp64_tol

pytestmark = pytest.mark.gpu

D, N = 64, 1 << 18
N_PSI, N_ROW, N_REL, N_AV, N_FE = 2048, 16384, 8192, 4096, 4096
RESID_KS = np.unique(np.concatenate([[1, 2, 1000, 20000], np.linspace(40000, N - 1, 12).astype(np.int64)]))
UP = np.array([1] * 32 + [0] * 32, dtype=np.int32)
ALPHA = np.eye(D)[0]


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def _log(msg):
    print(f"[c3 {time.strftime('%H:%M:%S')}] {msg}", flush=True)


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


@pytest.fixture(scope="module")
def c3(orc):
    """The kernel on the GPU and on the host, and every oracle reference."""
    _log("generating q")
    k = si.lognormal_kernel(D, N, si.CONFIG_SEEDS["c3"], device="cuda")
    qh = _np(k.q)
    ref = {"q": k.q, "qh": qh}
    t = time.time()
    ref["psi"] = orc.psi(qh[:N_PSI])
    _log(f"oracle psi prefix {N_PSI}: {time.time() - t:.1f} s")
    t = time.time()
    ref["row"] = orc.series_inverse_row(orc.e0_minus(qh[:N_ROW]), ALPHA)
    _log(f"oracle alpha-row {N_ROW}: {time.time() - t:.1f} s")
    t = time.time()
    ref["P"] = orc.transition(ref["psi"], qh[:N_PSI])
    ref["R"] = orc.reliability(qh[:N_REL], UP, ALPHA)
    ref["A"] = orc.availability(qh[:N_AV], UP, ALPHA)
    inD = np.zeros(D, dtype=np.int32)
    inD[D - 1] = 1
    ref["F"] = orc.first_entrance(qh[:N_FE], inD, ALPHA)[1]
    _log(f"oracle functionals: {time.time() - t:.1f} s")
    return ref


@pytest.fixture(scope="module")
def psis(mr, c3):
    out = {}
    for form in ("fp64", "mixed", "bf16x3"):
        _log(f"psi_inverse {form}")
        out[form] = mr.psi_inverse(c3["q"], form, check=True)
    torch.cuda.synchronize()
    return out


def _tol(form, n=N):
    return fp64_tol(n) if form == "fp64" else MIXED_TOL


@pytest.mark.parametrize("form", ["fp64", "mixed", "bf16x3"])
def test_c3_psi_prefix_and_alpha_row(mr, c3, psis, form):
    psi = psis[form]
    e_pre = _maxerr(_np(psi[:N_PSI]), c3["psi"])
    e_row = _maxerr(_np(psi[:N_ROW, 0, :]), c3["row"])
    _log(f"{form}: max|psi - oracle| prefix {N_PSI}: {e_pre:.3e}; alpha-row {N_ROW}: {e_row:.3e}")
    assert e_pre <= (FP64_TOL if form == "fp64" else MIXED_TOL)
    assert e_row <= (FP64_TOL if form == "fp64" else MIXED_TOL)


@pytest.mark.parametrize("form", ["fp64", "mixed", "bf16x3"])
def test_c3_sampled_residuals_over_the_horizon(mr, orc, c3, psis, form):
    t = time.time()
    rho = orc.residual_at(c3["qh"], _np(psis[form]), RESID_KS, e0_minus=True)
    per_k = np.max(np.abs(rho), axis=(1, 2))
    _log(f"{form}: direct residuals at {len(RESID_KS)} coefficients up to {RESID_KS[-1]} "
         f"({time.time() - t:.1f} s): max {per_k.max():.3e}")
    assert per_k.max() <= _tol(form)


@pytest.mark.parametrize("form", ["fp64", "mixed", "bf16x3"])
def test_c3_functionals(mr, c3, psis, form):
    """P = psi*Hbar is one transform product at length 2^19 over a recurrent
    psi, so each entry carries the product rounding of the whole horizon
    (bounded like psi by fp64_tol(n) in FP64; the product runs in FP64 in both
    forms).  Availability sums the |U| = 32 entries alpha P(k) 1_U, so its
    bound is |U| times P's.  Reliability and the first entrance come from the
    inverses of the transient blocks q_UU and q_CC and keep psi's bound."""
    psi, q = psis[form], c3["q"]
    P = mr.transition(psi, q)
    tol = FP64_TOL if form == "fp64" else MIXED_TOL
    p_tol = fp64_tol(N) if form == "fp64" else MIXED_TOL
    a_tol = int(UP.sum()) * p_tol
    e_P = _maxerr(_np(P[:N_PSI]), c3["P"])
    rows = float((P.sum(dim=2) - 1).abs().max())
    A = mr.availability(P, UP, ALPHA)
    del P
    R = mr.reliability(q, UP, ALPHA, precision=form)
    inD = [0] * (D - 1) + [1]
    _, F = mr.first_entrance(q, inD, ALPHA, precision=form)
    e_R = _maxerr(_np(R[:N_REL]), c3["R"])
    e_A = _maxerr(_np(A[:N_AV]), c3["A"])
    e_F = _maxerr(_np(F[:N_FE]), c3["F"])
    _log(f"{form}: P {e_P:.2e} (row sums {rows:.2e}), R {e_R:.2e}, A {e_A:.2e}, F {e_F:.2e}")
    assert e_P <= p_tol and e_A <= a_tol
    assert e_R <= tol and e_F <= tol
    assert rows <= _tol(form)


@pytest.mark.parametrize("form", ["mixed", "bf16x3"])
def test_c3_mixed_against_fp64_whole_horizon(psis, form):
    diff = float((psis[form] - psis["fp64"]).abs().max())
    _log(f"max|{form} - fp64| over the horizon: {diff:.3e}")
    assert diff <= MIXED_TOL
