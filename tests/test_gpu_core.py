"""GPU parity of the HIP path against the CPU FP64 oracle, element by element.

Every call goes through the C-ABI library (libmrinv.so) via the thin Python
binding.  Sizes span single-pass and multi-pass transform plans, ragged
(non-power-of-two) horizons, odd matrix dimensions (odd lane counts) and the
degenerate cases n = 1, d = 1.  Tolerance for FP64: max-abs error <= 1e-12
on the stochastic kernels; the mixed form: <= 1e-10.
"""
import numpy as np
import pytest
import torch

import smk_inputs as si

pytestmark = pytest.mark.gpu

from tolerances import FP64_TOL, MIXED_TOL, fp64_tol  # noqa: E402


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("d,n", [(1, 1), (1, 2), (2, 1), (4, 2), (3, 3), (4, 256), (5, 37), (2, 100),
                                 (7, 129), (16, 64), (3, 513), (6, 1000)])
def test_psi_fp64_matches_oracle(mr, orc, d, n):
    print(f"[psi fp64] d={d} n={n}", flush=True)
    q = si.weibull_kernel(d, n, 100 + d + n).q
    ref = orc.psi(q.numpy())
    got = _np(mr.psi_inverse(_gpu(q), check=True))
    assert _maxerr(got, ref) <= FP64_TOL


def test_psi_c1_config_and_transition(mr, orc):
    """Plain FP64 inversion, d = 4, n = 256, Weibull kernel, seed 0; psi and P."""
    k = si.weibull_kernel(4, 256, si.CONFIG_SEEDS["c1"])
    q = k.q.numpy()
    ref = orc.psi(q)
    psi = mr.psi_inverse(_gpu(q), check=True)
    assert _maxerr(_np(psi), ref) <= FP64_TOL
    P = _np(mr.transition(psi, _gpu(q)))
    Pref = orc.transition(ref, q)
    assert _maxerr(P, Pref) <= FP64_TOL
    assert np.max(np.abs(P.sum(axis=2) - 1.0)) <= 1e-13


@pytest.mark.parametrize("d,n", [(3, 5000), (2, 20000)])
def test_psi_two_pass_plans(mr, orc, d, n):
    """Horizons whose last Newton steps need two-pass transforms."""
    print(f"[psi two-pass] d={d} n={n}", flush=True)
    q = si.lognormal_kernel(d, n, 7 + d).q
    ref = orc.psi(q.numpy())
    got = _np(mr.psi_inverse(_gpu(q), check=True))
    assert _maxerr(got, ref) <= FP64_TOL


def test_psi_three_pass_geometric_closed_form(mr, orc):
    """n = 300000 (L = 2^19, three passes): Markov closed form at sampled k."""
    d, n = 3, 300000
    k = si.geometric_kernel(d, n, 31)
    got = mr.psi_inverse(k.q.cuda(), check=True)
    ks = np.array([0, 1, 2, 3, 100, 4097, 65536, 131071, 262144, n - 1])
    ref = orc.geometric_psi(k.params["M"], k.params["a"], ks)
    assert _maxerr(_np(got[torch.as_tensor(ks).cuda()]), ref) <= fp64_tol(n)


def test_psi_largest_d64_problem_closed_form(mr, orc):
    """The largest d = 64 FP64 inversion that fits one GPU with room to spare:
    a ragged horizon n = 2^20 - 4321 (last Newton step truncated, three-pass
    transforms at L = 2^20, about 171 GB of q, psi and workspace).  The Markov
    closed form at sampled k across the whole horizon, within the long-horizon
    FP64 bound."""
    d, n = 64, (1 << 20) - 4321
    torch.cuda.empty_cache()
    k = si.geometric_kernel(d, n, 37, device="cuda")
    got = mr.psi_inverse(k.q, check=True)
    ks = np.unique(np.concatenate([[0, 1, 2, 3, 4095, 4096, 65535, 524287, 524288, n - 2, n - 1],
                                   np.linspace(0, n - 1, 24).astype(int)]))
    ref = orc.geometric_psi(k.params["M"], k.params["a"], ks)
    e = _maxerr(_np(got[torch.as_tensor(ks).cuda()]), ref)
    print(f"[max] d={d} n={n}: {e:.3e}", flush=True)
    del got, k
    torch.cuda.empty_cache()
    assert e <= fp64_tol(n)


def test_padded_newton_meets_the_fp64_target_at_long_horizons(mr, orc):
    """The zero-padded Newton length (MRINV_FP64_PADDED) removes the
    wrap-around of the cyclic first product, whose rounding grows along a
    recurrent kernel's horizon: at n = 300000 the Markov closed form holds to
    the 1e-12 target, not only to the relaxed long-horizon bound."""
    d, n = 3, 300000
    k = si.geometric_kernel(d, n, 31)
    got = mr.psi_inverse(k.q.cuda(), "fp64_padded", check=True)
    ks = np.unique(np.concatenate([[0, 1, 2, 3, 100, 4097, 65536, 131071, 262144, n - 1],
                                   np.linspace(0, n - 1, 100).astype(int)]))
    ref = orc.geometric_psi(k.params["M"], k.params["a"], ks)
    e = _maxerr(_np(got[torch.as_tensor(ks).cuda()]), ref)
    print(f"[padded] n={n}: {e:.3e}", flush=True)
    assert e <= FP64_TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed", "bf16x3", "fp64_padded"])
def test_maximum_horizon_geometric_closed_form(mr, orc, precision):
    """The largest supported horizon, n = 2^21 (three-pass transforms up to
    L = 2^21, mixed sweeps at 2^22): Markov closed form at sampled k,
    including the last coefficient."""
    n, d = 1 << 21, 2   # MRINV_MAX_N
    k = si.geometric_kernel(d, n, 41)
    print(f"[max-horizon] d={d} n={n} {precision}", flush=True)
    got = mr.psi_inverse(k.q.cuda(), precision, check=True)
    ks = np.array([0, 1, 2, 5, 1000, 65537, 1 << 20, n - 2, n - 1])
    ref = orc.geometric_psi(k.params["M"], k.params["a"], ks)
    # At 2^21 the transform rounding of lengths up to 2^22 (2^23 padded) sets the
    # FP64 bound in both FP64 forms; the padded form removes the wrap-around
    # error only (see the n = 300000 test above).
    tol = {"fp64": fp64_tol(2 * n), "fp64_padded": fp64_tol(2 * n)}.get(precision, MIXED_TOL)
    e = _maxerr(_np(got[torch.as_tensor(ks).cuda()]), ref)
    print(f"[max-horizon] {precision}: {e:.3e} (bound {tol:.1e})", flush=True)
    assert e <= tol


def test_empty_and_oversized_horizons_are_rejected(mr):
    with pytest.raises((mr.MrinvError, ValueError)):
        mr.psi_inverse(torch.zeros((0, 3, 3), dtype=torch.float64).cuda())
    with pytest.raises(mr.MrinvError):
        mr.psi_inverse(torch.zeros(((1 << 21) + 1, 1, 1), dtype=torch.float64).cuda())
    mr.sync_status()


def test_prefix_exactness_and_causality(mr):
    """Proposition 2.3 on the GPU: the first n' coefficients do not depend on
    q(k >= n') and equal the horizon-n' inverse (within rounding)."""
    k = si.weibull_kernel(5, 3000, 41)
    q = k.q.cuda()
    full = mr.psi_inverse(q)
    q2 = q.clone()
    q2[1000:] *= 0.25
    part = mr.psi_inverse(q2)
    pre = mr.psi_inverse(q[:1000].contiguous())
    torch.cuda.synchronize()
    assert float((full[:1000] - part[:1000]).abs().max()) <= 1e-13
    assert float((full[:1000] - pre).abs().max()) <= 1e-13


def test_transpose_symmetry(mr):
    k = si.weibull_kernel(6, 777, 42)
    q = k.q.cuda()
    a = mr.psi_inverse(q)
    b = mr.psi_inverse(q.transpose(1, 2).contiguous())
    torch.cuda.synchronize()
    assert float((a - b.transpose(1, 2)).abs().max()) <= 1e-13


def test_series_inverse_general_A0(mr, orc):
    """A(0) != I exercises the Gauss-Jordan seed with pivoting."""
    rng = np.random.default_rng(3)
    d, n = 5, 300
    A = rng.standard_normal((n, d, d)) / (d * (1 + np.arange(n))[:, None, None] ** 2)
    A[0] = rng.standard_normal((d, d)) + 0.5 * np.eye(d)
    ref = orc.series_inverse_left(A)
    got = _np(mr.series_inverse(_gpu(A), check=True))
    assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("a0", ["diagonal", "permuted"])
def test_series_inverse_diagonal_and_permuted_A0(mr, orc, a0):
    """A diagonal A(0) with negative entries takes the Gauss-Jordan shortcut;
    a row-permuted diagonal one needs pivoting.  Both match the oracle, and
    the constant coefficient of the diagonal case is exactly 1 / a_rr."""
    rng = np.random.default_rng(5)
    d, n = 6, 200
    A = rng.standard_normal((n, d, d)) / (d * (1 + np.arange(n))[:, None, None] ** 2)
    diag = np.array([-2.0, 0.5, 3.0, -0.25, 7.0, 1.0])
    A[0] = np.diag(diag)
    if a0 == "permuted":
        A[0] = A[0][[2, 0, 1, 5, 3, 4]]
    ref = orc.series_inverse_left(A)
    got = _np(mr.series_inverse(_gpu(A), check=True))
    assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref)))
    if a0 == "diagonal":
        assert np.array_equal(got[0], np.diag(1.0 / diag))


@pytest.mark.parametrize("d,n,r", [(4, 100, 3), (5, 257, 1), (3, 64, 6)])
def test_apply_matches_oracle(mr, orc, d, n, r):
    rng = np.random.default_rng(d * n + r)
    q = si.weibull_kernel(d, n, 5).q.numpy()
    psi = orc.psi(q)
    L = rng.uniform(0, 1, (n, d, r))
    ref = orc.conv(psi, L)
    got = _np(mr.markov_renewal_apply(_gpu(psi), _gpu(L)))
    assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("d,n", [(3, 50), (8, 600), (5, 1)])
def test_transition_matches_oracle(mr, orc, d, n):
    q = si.weibull_kernel(d, n, 9).q.numpy()
    psi = orc.psi(q)
    ref = orc.transition(psi, q)
    got = _np(mr.transition(_gpu(psi), _gpu(q)))
    assert _maxerr(got, ref) <= FP64_TOL
    hb = _np(mr.survival(_gpu(q)))
    assert _maxerr(hb, orc.hbar(q)) <= 1e-14


def test_paper_first_entrance_example(mr, orc):
    """Section 5.1 first restoration (Poisson 8, 5, 10, 7; D = {1}, C = {2, 3},
    alpha_C = (1, 0), N = 128): closed-form mass and F(N-1) = 1."""
    from scipy.stats import poisson
    n = 128
    q = si.paper_three_state_poisson(n).q
    g, F = mr.first_entrance(q.cuda(), [1, 0, 0], [0.0, 1.0, 0.0])
    t = np.arange(n)
    ref = 0.2 * np.where(t >= 1, poisson.pmf(t - 1, 5.0), 0) + 0.8 * np.where(t >= 2, poisson.pmf(t - 2, 17.0), 0)
    assert _maxerr(_np(g), ref) <= 1e-15 * 10
    assert abs(_np(F)[-1] - 1.0) <= 1e-14



def test_paper_horizon_scaling_accuracy(mr, orc):
    """The paper's horizon-scaling model (Section 5.1; fixture
    golden/inverse_accuracy.txt) at N = 128, 512, 2048: the library's FP64
    inverse is at least as accurate as the FFT-Newton figures the paper
    prints: scaled discrepancy d_N from the coefficient recursion (the
    oracle's right recursion, the paper's eq. (inverse-recursion)) and the
    left and right residuals in the norm ||.||_{1,N} (Section 2), both formed
    by the oracle with direct convolutions.  On the state-dimension model
    (s = 2, 4, 6, 8, N = 256) the residuals stay within the top of the range
    the paper prints for both experiments."""
    import paper_fixtures as pf

    fx = pf.read_blocks("inverse_accuracy.txt")
    for N, dN, left, right in fx["fft_newton"]:
        q = si.paper_three_state_gamma(int(N)).q.numpy()
        psi = _np(mr.psi_inverse(_gpu(q)))
        got_d = orc.scaled_discrepancy(psi, orc.psi_right(q))
        rL, rR = orc.residuals(orc.e0_minus(q), psi)
        got = (got_d, orc.norm_1N(rL), orc.norm_1N(rR))
        print(f"N={N}: d_N={got[0]:.3g} left={got[1]:.3g} right={got[2]:.3g}", flush=True)
        for g, v in zip(got, (dN, left, right)):
            assert g <= float(v), (N, g, v)
    # State-dimension experiment: residuals within the top of the printed range.
    top = float(fx["residual_range"][0][1])
    for s_, N in fx["state_dimension"]:
        q = si.paper_uniform_poisson(int(s_), int(N)).q.numpy()
        psi = _np(mr.psi_inverse(_gpu(q)))
        rL, rR = orc.residuals(orc.e0_minus(q), psi)
        print(f"s={s_}: left={orc.norm_1N(rL):.3g} right={orc.norm_1N(rR):.3g}", flush=True)
        assert max(orc.norm_1N(rL), orc.norm_1N(rR)) <= top, (s_, top)

def test_reliability_and_availability_match_oracle(mr, orc):
    d, n = 6, 400
    q = si.weibull_kernel(d, n, 12).q.numpy()
    up = [1, 1, 1, 0, 0, 0]
    alpha = np.eye(d)[0]
    R = _np(mr.reliability(_gpu(q), up, alpha))
    assert _maxerr(R, orc.reliability(q, np.array(up), alpha)) <= FP64_TOL
    psi = mr.psi_inverse(_gpu(q))
    P = mr.transition(psi, _gpu(q))
    A = _np(mr.availability(P, up, alpha))
    assert _maxerr(A, orc.availability(q, np.array(up), alpha)) <= FP64_TOL


def test_geometric_functionals_closed_form(mr, orc):
    d, n = 8, 2048
    k = si.geometric_kernel(d, n, 13)
    M = k.params["M"]
    q = k.q.cuda()
    up = [1] * 4 + [0] * 4
    alpha = np.eye(d)[0]
    psi = mr.psi_inverse(q)
    P = mr.transition(psi, q)
    ks = np.array([0, 1, 5, 100, 1000, n - 1])
    assert _maxerr(_np(P)[ks], orc.geometric_P(M, ks)) <= FP64_TOL
    A = _np(mr.availability(P, up, alpha))
    Aref = np.array([alpha @ np.linalg.matrix_power(M, int(t)) @ np.array(up, float) for t in ks])
    assert _maxerr(A[ks], Aref) <= FP64_TOL
    R = _np(mr.reliability(q, up, alpha))
    Rref = np.array([alpha[:4] @ np.linalg.matrix_power(M[:4, :4], int(t)) @ np.ones(4) for t in ks])
    assert _maxerr(R[ks], Rref) <= FP64_TOL


@pytest.mark.parametrize("d,n", [(4, 256), (8, 4096), (3, 1000), (16, 2048)])
@pytest.mark.parametrize("precision", ["mixed", "bf16x3"])
def test_mixed_precision_matches_oracle(mr, orc, d, n, precision):
    print(f"[psi {precision}] d={d} n={n}", flush=True)
    q = si.lognormal_kernel(d, n, 200 + d).q
    ref = orc.psi(q.numpy())
    got = _np(mr.psi_inverse(_gpu(q), precision=precision, check=True))
    assert _maxerr(got, ref) <= MIXED_TOL


def test_psi_backward_matches_oracle_adjoint(mr, orc):
    rng = np.random.default_rng(4)
    d, n = 4, 200
    q = si.weibull_kernel(d, n, 14).q.numpy()
    psi = orc.psi(q)
    pb = rng.standard_normal((n, d, d))
    ref = orc.adjoint(psi, pb)
    got = _np(mr.psi_inverse_backward(_gpu(psi), _gpu(pb)))
    assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("d", [12, 17, 32, 33])
def test_psi_backward_transposed_products_match_oracle(mr, orc, d):
    """The adjoint's products with a transposed operand on the matrix cores
    (mfma = 1, 2) and on the vector kernel (mfma = 0) against the oracle."""
    rng = np.random.default_rng(40 + d)
    n = 150
    q = si.weibull_kernel(d, n, 60 + d).q.numpy()
    psi = orc.psi(q)
    pb = rng.standard_normal((n, d, d))
    ref = orc.adjoint(psi, pb)
    base = mr.get_tuning()
    try:
        for mode in (0, 1, 2):
            mr.set_tuning(mfma=mode)
            got = _np(mr.psi_inverse_backward(_gpu(psi), _gpu(pb)))
            assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref))), mode
    finally:
        mr.set_tuning(**base)


@pytest.mark.parametrize("w,n,reverse", [(1, 1, 0), (1, 5000, 1), (16, 1025, 0), (31, 3000, 1), (64, 2049, 0)])
def test_time_scans(mr, w, n, reverse):
    """Survival sequence H-bar (a scan over time of d lanes, Section 4.1) and
    the cumulative contraction against numpy cumulative sums."""
    rng = np.random.default_rng(w + n)
    if reverse == 0:
        q = rng.random((n, w, w)) / (w * n)
        q[0] = 0.0
        hb = _np(mr.survival(_gpu(q)))
        ref = 1.0 - np.cumsum(q.sum(axis=2), axis=0)
        assert hb.shape == (n, w)
        assert _maxerr(hb, ref) <= 1e-13
    X = rng.standard_normal((n, w, 2))
    u = rng.standard_normal(w)
    v = rng.standard_normal(2)
    out = _np(mr.contract(_gpu(X), torch.tensor(u), torch.tensor(v), cumulative=True))
    ref = np.cumsum(np.einsum("kij,i,j->k", X, u, v))
    assert _maxerr(out, ref) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    if reverse:
        ob = rng.standard_normal(n)
        Xb = _np(mr.contract_backward(_gpu(ob), w, 2, u, v, cumulative=True))
        rs = np.cumsum(ob[::-1])[::-1]
        refb = rs[:, None, None] * u[None, :, None] * v[None, None, :]
        assert _maxerr(Xb, refb) <= 1e-10 * max(1.0, np.max(np.abs(refb)))


def test_apply_backward_matches_direct(mr, orc):
    """psi_bar(l) = sum_k M_bar(k) L(k-l)^T and L_bar(j) = sum_l psi(l)^T M_bar(l+j),
    evaluated with the oracle's direct convolution on reversed sequences."""
    rng = np.random.default_rng(5)
    d, n, r = 3, 150, 2
    psi = rng.standard_normal((n, d, d))
    L = rng.standard_normal((n, d, r))
    Mb = rng.standard_normal((n, d, r))
    pb, lb = mr.markov_renewal_apply_backward(_gpu(psi), _gpu(L), _gpu(Mb))
    rev = lambda x: x[::-1].copy()
    pref = rev(orc.conv(rev(Mb), np.ascontiguousarray(L.transpose(0, 2, 1))))
    lref = rev(orc.conv(np.ascontiguousarray(psi.transpose(0, 2, 1)), rev(Mb)))
    assert _maxerr(_np(pb), pref) <= 1e-10
    assert _maxerr(_np(lb), lref) <= 1e-10


def test_autograd_transition_and_functionals_fd(mr):
    """Gradient of sum_k A(k) through PsiInverse, Transition and Contract
    against a central finite difference along a random direction."""
    d, n = 4, 128
    k = si.weibull_kernel(d, n, 15)
    q0 = k.q.cuda()
    up = torch.tensor([1.0, 1.0, 0.0, 0.0], dtype=torch.float64)
    alpha = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=torch.float64)

    def loss(q):
        psi = mr.PsiInverse.apply(q)
        P = mr.Transition.apply(psi, q)
        return mr.Contract.apply(P, alpha, up).sum()

    q = q0.clone().requires_grad_(True)
    loss(q).backward()
    g = q.grad.detach()
    torch.manual_seed(0)
    dq = torch.randn_like(q0)
    dq[0] = 0
    h = 1e-6
    with torch.no_grad():
        fd = (loss(q0 + h * dq) - loss(q0 - h * dq)) / (2 * h)
    an = float((g * dq).sum())
    assert abs(an - float(fd)) <= 1e-6 * max(1.0, abs(an))


def test_singular_a0_is_reported(mr):
    d, n = 3, 16
    A = torch.zeros((n, d, d), dtype=torch.float64)
    A[0] = torch.diag(torch.tensor([1.0, 0.0, 2.0]))
    out = mr.series_inverse(A.cuda())
    with pytest.raises(mr.MrinvError) as e:
        mr.sync_status()
    assert e.value.status == 2
    assert torch.isnan(out[0]).all()


def test_nonfinite_is_reported(mr):
    q = si.weibull_kernel(3, 64, 16).q
    q[10, 1, 2] = float("nan")
    mr.psi_inverse(q.cuda())
    with pytest.raises(mr.MrinvError) as e:
        mr.sync_status()
    assert e.value.status == 3


def test_argument_errors(mr):
    with pytest.raises(mr.MrinvError):
        mr.psi_inverse(torch.zeros((4, 65, 65), dtype=torch.float64).cuda())
    with pytest.raises(mr.MrinvError):
        mr.psi_inverse(torch.zeros((4, 3, 3), dtype=torch.float32).cuda())
    with pytest.raises(mr.MrinvError):
        mr.psi_inverse(torch.zeros((4, 3, 3), dtype=torch.float64))
    mr.sync_status()


def test_deterministic_reruns(mr):
    q = si.weibull_kernel(7, 3333, 17).q.cuda()
    a = mr.psi_inverse(q)
    b = mr.psi_inverse(q)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "bf16x3", "fp64_padded"])
def test_batched_matches_single_calls_and_oracle(mr, orc, precision):
    """Uneven batch (odd and even d, ragged n, n = 1): each problem equals the
    single-problem call (same kernels, same plans) and the oracle."""
    specs = [(1, 5), (2, 1), (3, 37), (5, 300), (8, 1000), (16, 513), (17, 64), (31, 200), (33, 129), (48, 70),
             (4, 2048), (6, 3000)]
    qs = [si.family_kernel("weibull" if i % 2 else "lognormal", d, n, 300 + i).q.cuda()
          for i, (d, n) in enumerate(specs)]
    outs = mr.psi_inverse_batched(qs, precision)
    mr.sync_status()
    tol = FP64_TOL if precision.startswith("fp64") else MIXED_TOL
    for (d, n), q, o in zip(specs, qs, outs):
        single = mr.psi_inverse(q, precision)
        torch.cuda.synchronize()
        assert torch.equal(o, single), (d, n)
        ref = orc.psi(q[: min(n, 600)].cpu().numpy())
        assert _maxerr(_np(o[: min(n, 600)]), ref) <= tol, (d, n)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_wide_problems_match_single_calls_and_oracle(mr, orc, precision):
    """Problems with padded d = 64 (even and odd d) in one batch, long enough
    for transform steps: the batched products take the same three-product,
    two-waves-per-strip kernels as the single calls (bitwise equal), and both
    match the oracle on a prefix."""
    specs = [(64, 1500), (57, 1100), (50, 700), (20, 1500)]
    qs = [si.family_kernel("lognormal" if i % 2 else "weibull", d, n, 900 + i).q.cuda()
          for i, (d, n) in enumerate(specs)]
    outs = mr.psi_inverse_batched(qs, precision)
    mr.sync_status()
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for (d, n), q, o in zip(specs, qs, outs):
        single = mr.psi_inverse(q, precision)
        torch.cuda.synchronize()
        assert torch.equal(o, single), (d, n)
        ref = orc.psi(q[:300].cpu().numpy())
        assert _maxerr(_np(o[:300]), ref) <= tol, (d, n)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("d", [6, 64])
def test_graph_replays_match_eager(mr, precision, d):
    """With graph recording on, repeated calls with the same pointers replay
    one HIP graph.  Every replay, with eager work and new input values in
    between, must equal the eager (unrecorded) result bitwise.  At d = 64 the
    FP64 products are the streamed kernel (a grid of resident workgroups)."""
    import ctypes
    n = 3000
    prec = mr._PREC[precision]
    q = si.weibull_kernel(d, n, 61).q.cuda()
    q2 = si.lognormal_kernel(d, n, 62).q.cuda()
    out = torch.empty_like(q)
    ws = torch.empty(mr.workspace_size("psi_inverse", d, n, 0, precision), dtype=torch.uint8, device="cuda")
    dev = q.device
    L = mr.lib()

    def call():
        mr._check(L.mrinv_psi_inverse(mr._handle(dev), ctypes.c_void_p(q.data_ptr()), d, n, prec,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel()))

    base = mr.get_tuning()
    try:
        mr.set_tuning(use_graph=0)
        call()
        ref1 = out.clone()
        saved = q.clone()
        q.copy_(q2)
        call()
        ref2 = out.clone()
        q.copy_(saved)
        mr.set_tuning(use_graph=1)
        for rep in range(4):
            out.fill_(float("nan"))          # eager work between replays
            torch.cuda.synchronize()
            call()
            torch.cuda.synchronize()
            assert torch.equal(out, ref1), rep
        q.copy_(q2)                          # same pointers, new values
        call()
        torch.cuda.synchronize()
        assert torch.equal(out, ref2)
        mr.sync_status()
    finally:
        mr.set_tuning(**base)


@pytest.mark.parametrize("d", [9, 12, 16, 24, 25, 31, 32, 40, 47, 48, 57, 63, 64])
def test_matrix_core_products_match_oracle(mr, orc, d):
    """Square frequency-domain products on the matrix cores (mfma = 2), on
    the vector kernels (mfma = 0) and the default choice (mfma = 1), in FP64,
    the padded FP64 Newton and both mixed forms (float32 and split-BF16
    products), odd and even d, all against the oracle; the two FP64 kernels
    agree to rounding."""
    n = 300
    print(f"[mfma] d={d} n={n}", flush=True)
    q = si.family_kernel("lognormal" if d % 2 else "weibull", d, n, 700 + d).q
    ref = orc.psi(q.numpy())
    qg = _gpu(q)
    base = mr.get_tuning()
    got = {}
    try:
        for mode in (0, 1, 2):
            mr.set_tuning(mfma=mode)
            for prec in ("fp64", "mixed", "bf16x3", "fp64_padded"):
                o = _np(mr.psi_inverse(qg, prec, check=True))
                tol = FP64_TOL if prec.startswith("fp64") else MIXED_TOL
                assert _maxerr(o, ref) <= tol, (mode, prec)
                got[mode, prec] = o
    finally:
        mr.set_tuning(**base)
    assert _maxerr(got[0, "fp64"], got[2, "fp64"]) <= 1e-13


@pytest.mark.parametrize("d,n", [(16, 8192), (33, 2048), (64, 1500), (4, 40000)])
def test_lanes_per_workgroup_do_not_change_the_bits(mr, d, n):
    """The transform passes compute the same bits whatever their lanes per
    workgroup (8, 16 or 32, or the automatic choice 0; 16 takes the half-lane
    LDS tile for 256- and 512-row FP64 passes), so every lane setting gives
    one result."""
    q = _gpu(si.family_kernel("weibull", d, n, 60 + d).q)
    base = mr.get_tuning()
    outs = {}
    try:
        for lanes in (0, 8, 16, 32):
            mr.set_tuning(lanes_fp64=lanes, lanes_fp32=lanes)
            for prec in ("fp64", "mixed"):
                outs[lanes, prec] = _np(mr.psi_inverse(q, prec, check=True))
    finally:
        mr.set_tuning(**base)
    for prec in ("fp64", "mixed"):
        for lanes in (0, 8, 32):
            assert np.array_equal(outs[lanes, prec], outs[16, prec]), (lanes, prec)


@pytest.mark.parametrize("tuning", [dict(mfma=2), dict(seed_m0=16, direct_m=0), dict(direct_m=1024, mfma=0)])
def test_matrix_core_batched_matches_single_calls(mr, orc, tuning):
    """Under non-default tunings (all products on the matrix cores; recursion
    seed and transforms only; direct steps up to 1024 with vector products)
    the batched call, planned and sized for the handle's tuning, still equals
    the single-problem calls bitwise (same kernel bodies) and the oracle."""
    specs = [(9, 100), (16, 257), (23, 64), (32, 130), (41, 40), (64, 33), (5, 77)]
    qs = [si.family_kernel("weibull", d, n, 800 + i).q.cuda() for i, (d, n) in enumerate(specs)]
    base = mr.get_tuning()
    try:
        mr.set_tuning(**tuning)
        for prec in ("fp64", "mixed"):
            outs = mr.psi_inverse_batched(qs, prec)
            mr.sync_status()
            for (d, n), q, o in zip(specs, qs, outs):
                single = mr.psi_inverse(q, prec)
                torch.cuda.synchronize()
                assert torch.equal(o, single), (prec, d, n)
                ref = orc.psi(q.cpu().numpy())
                assert _maxerr(_np(o), ref) <= (FP64_TOL if prec == "fp64" else MIXED_TOL), (prec, d, n)
    finally:
        mr.set_tuning(**base)


@pytest.mark.parametrize("d", [1, 3, 4, 16, 17, 33, 64])
def test_direct_steps_match_oracle(mr, orc, d):
    """Newton steps formed directly in the time domain (direct_m), none of
    them (0), the automatic choice (-1) and all of them, with and without the
    recursion seed, FP64 and mixed, against the oracle."""
    n = 200 if d <= 33 else 90
    print(f"[direct] d={d} n={n}", flush=True)
    q = si.family_kernel("weibull" if d % 2 == 0 else "lognormal", d, n, 900 + d).q
    ref = orc.psi(q.numpy())
    qg = _gpu(q)
    base = mr.get_tuning()
    try:
        for direct_m, seed in ((0, 1), (-1, 1), (65536, 1), (65536, 16), (64, 8)):
            mr.set_tuning(direct_m=direct_m, seed_m0=seed)
            for prec in ("fp64", "mixed", "bf16x3", "fp64_padded"):
                o = _np(mr.psi_inverse(qg, prec, check=True))
                tol = FP64_TOL if prec == "fp64" else MIXED_TOL
                assert _maxerr(o, ref) <= tol, (direct_m, seed, prec)
    finally:
        mr.set_tuning(**base)


def test_direct_steps_series_inverse_general_a0(mr, orc):
    """series_inverse with a general A(0) through direct steps only."""
    d, n = 5, 120
    rng = np.random.default_rng(41)
    A = rng.standard_normal((n, d, d)) / (d * (1 + np.arange(n))[:, None, None] ** 2)
    A[0] = rng.standard_normal((d, d)) + 0.5 * np.eye(d)
    ref = orc.series_inverse_left(A)
    base = mr.get_tuning()
    try:
        mr.set_tuning(direct_m=65536)
        got = _np(mr.series_inverse(_gpu(A), check=True))
    finally:
        mr.set_tuning(**base)
    assert _maxerr(got, ref) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_keeps_a_valid_tuning(mr, orc, precision):
    """The autotuner's choice is a valid tuning (it can be set again), stays
    in the handle, and the inverse under it still matches the oracle."""
    d, n = 12, 3000
    q = si.family_kernel("weibull", d, n, 88).q
    ref = orc.psi(q.numpy())
    qg = _gpu(q)
    base = mr.get_tuning()
    try:
        chosen = mr.autotune(qg, precision)
        assert set(chosen) == set(base)
        assert chosen == mr.get_tuning()
        assert chosen["lanes_fp64"] in (0, 8, 16, 32) and chosen["lanes_fp32"] in (0, 8, 16, 32)
        assert 5 <= chosen["lgp_max"] <= 9 and chosen["mfma"] in (0, 1, 2)
        mr.set_tuning(**chosen)
        got = _np(mr.psi_inverse(qg, precision, check=True))
        tol = FP64_TOL if precision == "fp64" else MIXED_TOL
        assert _maxerr(got, ref) <= tol
    finally:
        mr.set_tuning(**base)


def test_residual_norms_match_oracle(mr, orc):
    """Residual diagnostics (Proposition 2.6): the library's FFT-based sums of
    ||e0 - A*X||_F and ||e0 - X*A||_F and max |e0 - A*X| against the oracle's
    direct convolutions, on a perturbed inverse so the residuals are far above
    rounding."""
    d, n = 5, 300
    q = si.family_kernel("weibull", d, n, 71).q
    psi = orc.psi(q.numpy())
    X = psi + 1e-6 * np.random.default_rng(3).standard_normal(psi.shape)
    rl, rr = orc.residuals(orc.e0_minus(q.numpy()), X)
    ref = (float(np.sum(np.linalg.norm(rl, axis=(1, 2)))), float(np.sum(np.linalg.norm(rr, axis=(1, 2)))),
           float(np.max(np.abs(rl))))
    got = mr.residual_norms(_gpu(q), _gpu(X))
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-8 * r, (got, ref)


def test_kernel_timing_records_every_launch(mr):
    """Timed launches (events stamped by the kernels' own dispatch packets)
    change no result, and their summed execution times fit inside the wall
    time of the calls they cover."""
    import ctypes

    class Stat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 96), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                    ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]

    L = mr.lib()
    L.mrinv_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.mrinv_set_timing.restype = ctypes.c_int
    L.mrinv_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stat), ctypes.c_int]
    L.mrinv_kernel_stats.restype = ctypes.c_int
    dev = torch.device("cuda:0")
    h = mr._handle(dev)
    q = _gpu(si.family_kernel("weibull", 16, 8192, 77).q)
    plain = _np(mr.psi_inverse(q, "fp64", check=True))
    calls = 3
    assert L.mrinv_set_timing(h, 1) == 0
    try:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        outs = [mr.psi_inverse(q, "fp64") for _ in range(calls)]
        t1.record()
        torch.cuda.synchronize()
        wall_ms = t0.elapsed_time(t1)
        buf = (Stat * 64)()
        k = L.mrinv_kernel_stats(h, buf, 64)
    finally:
        L.mrinv_set_timing(h, 0)
    assert 0 < k <= 64
    stats = [buf[i] for i in range(k)]
    names = [s.name.decode() for s in stats]
    assert any(n.startswith("fft_pass") for n in names), names
    assert any(n.startswith("freq_gemm") for n in names), names
    for s in stats:
        assert s.launches > 0 and s.launches % calls == 0, (s.name, s.launches)
        assert 0.0 < s.total_ms < wall_ms, (s.name, s.total_ms, wall_ms)
    assert sum(s.total_ms for s in stats) <= wall_ms
    for o in outs:
        assert np.array_equal(_np(o), plain)
