"""FFT-Gauss-Jordan inversion over the truncated series ring (Appendix,
Gauss-Jordan paragraph), through the C-ABI: element-by-element parity with
the oracle's recursion (the inverse is unique, Theorem 2.1 / Proposition
2.3), agreement with the Newton path, pivoting, the paper's accuracy rows for
this method, and a singular A(0)."""
import numpy as np
import pytest
import torch

import paper_fixtures as pf
import smk_inputs as si
from tolerances import FP64_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("d,n", [(1, 1), (1, 300), (2, 2), (3, 37), (4, 256), (5, 1000), (8, 513), (17, 200)])
def test_gj_psi_matches_oracle(mr, orc, d, n):
    print(f"[gj] psi d={d} n={n}", flush=True)
    q = si.weibull_kernel(d, n, 400 + d + n).q.numpy()
    got = _np(mr.series_inverse_gj(_gpu(q), check=True, e0_minus=True))
    assert _maxerr(got, orc.psi(q)) <= FP64_TOL
    newton = _np(mr.psi_inverse(_gpu(q)))
    assert _maxerr(got, newton) <= FP64_TOL


@pytest.mark.parametrize("a0", ["permuted", "general"])
def test_gj_general_a0_needs_pivoting(mr, orc, a0):
    """A(0) whose leading entries are zero (a permutation) or small forces row
    swaps; the result is still the oracle's unique inverse."""
    rng = np.random.default_rng(410)
    d, n = 5, 300
    A = rng.standard_normal((n, d, d)) / (d * np.arange(1, n + 1)[:, None, None] ** 1.5)
    if a0 == "permuted":
        A[0] = np.eye(d)[[3, 0, 4, 1, 2]] * np.array([2.0, 1.5, 1.0, 0.5, 3.0])[:, None]
    else:
        A[0] = rng.standard_normal((d, d)) + 0.5 * np.eye(d)
        A[0, 0, 0] = 1e-3
    got = _np(mr.series_inverse_gj(_gpu(A), check=True))
    ref = orc.series_inverse_left(A)
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert _maxerr(got, ref) <= 1e-12 * scale
    assert _maxerr(got, _np(mr.series_inverse(_gpu(A)))) <= 1e-12 * scale


def test_gj_paper_accuracy_rows(mr, orc):
    """The paper's FFT-Gauss-Jordan rows (Section 5.1 accuracy table, fixture
    golden/inverse_accuracy.txt): the left/right residuals in ||.||_{1,N},
    formed by the oracle with direct convolutions, are no larger than the
    printed values, and the scaled discrepancy from the coefficient recursion
    (two FP64 computations compared at the rounding level) is within twice
    the printed one."""
    fx = pf.read_blocks("inverse_accuracy.txt")
    for N, dN, left, right in fx["fft_gauss_jordan"]:
        q = si.paper_three_state_gamma(int(N)).q.numpy()
        psi = _np(mr.series_inverse_gj(_gpu(q), check=True, e0_minus=True))
        got_d = orc.scaled_discrepancy(psi, orc.psi_right(q))
        rL, rR = orc.residuals(orc.e0_minus(q), psi)
        got = (got_d, orc.norm_1N(rL), orc.norm_1N(rR))
        print(f"[gj] N={N}: d_N={got[0]:.3g} left={got[1]:.3g} right={got[2]:.3g}", flush=True)
        assert got[0] <= 2 * float(dN), (N, got[0], dN)
        for g, v in zip(got[1:], (left, right)):
            assert g <= float(v), (N, g, v)


def test_gj_singular_a0_is_reported(mr):
    d, n = 3, 40
    A = np.zeros((n, d, d))
    A[0] = np.diag([1.0, 0.0, 2.0])
    A[1] = 0.1
    with pytest.raises(mr.MrinvError) as ei:
        mr.series_inverse_gj(_gpu(A), check=True)
    assert ei.value.status == 2
