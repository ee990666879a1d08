"""Pins of the CPU FP64 oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own formulas.

Each test names what pins it: a brute-force enumeration, a closed form, an
exact identity, a library routine, or a worked example printed in the paper.
"""
from fractions import Fraction

import numpy as np
import pytest

import paper_fixtures as pf
import smk_inputs as si
from oracle import exact


def _rand_series(rng, n, d, a0_scale=1.0):
    A = rng.standard_normal((n, d, d)) / (d * np.arange(1, n + 1)[:, None, None])
    A[0] = np.eye(d) * 2.0 + a0_scale * rng.standard_normal((d, d)) * 0.3
    return A


def test_gj_inverse_matches_library(orc):
    rng = np.random.default_rng(10)
    for d in (1, 2, 5, 17, 64):
        A = rng.standard_normal((d, d)) + d * np.eye(d) * 0.1
        assert np.allclose(orc.gj_inverse(A), np.linalg.inv(A), rtol=1e-10, atol=1e-12)


def test_gj_singular_detected(orc):
    A = np.diag([1.0, 0.0, 2.0])
    with pytest.raises(orc.SingularError):
        orc.gj_inverse(A)
    S = np.zeros((4, 3, 3))
    S[0] = A
    with pytest.raises(orc.SingularError):
        orc.series_inverse_left(S)


def test_left_and_right_recursions_agree(orc):
    """Left recursion (from A*X = e0) and the paper's right recursion (from
    X*A = e0) are two definitions of the unique two-sided inverse (Thm 2.1)."""
    rng = np.random.default_rng(1)
    for d, n in ((1, 30), (3, 50), (6, 40)):
        A = _rand_series(rng, n, d)
        L = orc.series_inverse_left(A)
        R = orc.series_inverse_right(A)
        assert np.max(np.abs(L - R)) <= 1e-13 * max(1.0, np.max(np.abs(L)))


@pytest.mark.parametrize("d,n", [(1, 9), (2, 8), (3, 7)])
def test_exact_path_enumeration(orc, d, n):
    """psi = sum_m q^(m), enumerated over state paths and compositions in
    exact rationals (Theorem 2.1 Neumann form / renewal-sequence identity)."""
    rng = np.random.default_rng(100 + d)
    qf = exact.random_rational_kernel(d, n, rng)
    ex = exact.psi_paths(qf)
    q = np.array([[[float(x) for x in row] for row in mat] for mat in qf])
    got = orc.psi(q)
    exf = np.array([[[float(x) for x in row] for row in mat] for mat in ex])
    assert np.max(np.abs(got - exf)) <= 1e-15


def test_exact_enumeration_small_hand_case():
    """Hand check of the enumerator itself: d = 1, q(1) = 1/2, q(2) = 1/3.
    psi(1) = 1/2, psi(2) = q(2) + q(1)^2 = 1/3 + 1/4."""
    q = [[[Fraction(0)]], [[Fraction(1, 2)]], [[Fraction(1, 3)]]]
    ps = exact.psi_paths(q)
    assert ps[1][0][0] == Fraction(1, 2)
    assert ps[2][0][0] == Fraction(7, 12)


def test_geometric_closed_form(orc):
    """Geometric sojourns make the process a Markov chain with one-step matrix
    M = diag(a) + diag(1-a) p.  Then P(k) = M^k and psi(k) = M^(k-1)(M - diag(a))
    for k >= 1 (a jump lands at time k), psi(0) = I."""
    d, n = 5, 80
    k = si.geometric_kernel(d, n, 2)
    q = k.q.numpy()
    M, a = k.params["M"], k.params["a"]
    ps = orc.psi(q)
    ref = np.empty((n, d, d))
    ref[0] = np.eye(d)
    Mk = np.eye(d)
    for t in range(1, n):
        ref[t] = Mk @ (M - np.diag(a))
        Mk = Mk @ M
    assert np.max(np.abs(ps - ref)) <= 1e-14
    P = orc.transition(ps, q)
    Pref = np.array([np.linalg.matrix_power(M, t) for t in range(n)])
    assert np.max(np.abs(P - Pref)) <= 1e-13


def test_geometric_functionals_closed_form(orc):
    """Markov case: availability alpha M^k 1_U, reliability alpha_U M_UU^k 1_U,
    first entrance F_D(k) = 1 - alpha_C M_CC^k 1_C."""
    d, n = 6, 70
    k = si.geometric_kernel(d, n, 7)
    q = k.q.numpy()
    M = k.params["M"]
    up = np.array([1, 1, 1, 0, 0, 0])
    alpha = np.zeros(d)
    alpha[0] = 1.0
    A = orc.availability(q, up, alpha)
    Aref = np.array([alpha @ np.linalg.matrix_power(M, t) @ up for t in range(n)])
    assert np.max(np.abs(A - Aref)) <= 1e-13
    R = orc.reliability(q, up, alpha)
    MUU = M[:3, :3]
    Rref = np.array([alpha[:3] @ np.linalg.matrix_power(MUU, t) @ np.ones(3) for t in range(n)])
    assert np.max(np.abs(R - Rref)) <= 1e-13
    inD = np.zeros(d, dtype=int)
    inD[d - 1] = 1
    _, F = orc.first_entrance(q, inD, alpha)
    MCC = M[: d - 1, : d - 1]
    Fref = np.array([1 - alpha[: d - 1] @ np.linalg.matrix_power(MCC, t) @ np.ones(d - 1) for t in range(n)])
    assert np.max(np.abs(F - Fref)) <= 1e-13


def test_scalar_geometric(orc):
    """d = 1, f(k) = (1-a)a^(k-1): every step is a renewal with probability 1-a."""
    a, n = 0.7, 50
    q = np.zeros((n, 1, 1))
    q[1:, 0, 0] = (1 - a) * a ** np.arange(n - 1)
    ps = orc.psi(q)
    assert abs(ps[0, 0, 0] - 1.0) == 0.0
    assert np.max(np.abs(ps[1:, 0, 0] - (1 - a))) <= 1e-15


def test_unit_sojourn_gives_matrix_powers(orc):
    """q(k) = 0 except q(1) = B: psi = sum_m q^(m) has psi(k) = B^k."""
    rng = np.random.default_rng(3)
    d, n = 4, 25
    B = rng.uniform(0, 0.3, (d, d))
    q = np.zeros((n, d, d))
    q[1] = B
    ps = orc.psi(q)
    ref = np.array([np.linalg.matrix_power(B, t) for t in range(n)])
    assert np.max(np.abs(ps - ref)) <= 1e-15


def test_conv_against_library_convolve(orc):
    """(A*B)_ij = sum_t convolve(A_it, B_tj)[:n] (numpy.convolve per entry)."""
    rng = np.random.default_rng(4)
    n, ra, m, cb = 37, 3, 4, 2
    A = rng.standard_normal((n, ra, m))
    B = rng.standard_normal((n, m, cb))
    C = orc.conv(A, B)
    ref = np.zeros((n, ra, cb))
    for i in range(ra):
        for j in range(cb):
            for t in range(m):
                ref[:, i, j] += np.convolve(A[:, i, t], B[:, t, j])[:n]
    assert np.max(np.abs(C - ref)) <= 1e-12


def test_transition_row_sums_exact_identity(orc):
    """P 1 = s0 * psi * (e0 - q) 1 = 1 for ANY q with q(0) = 0 (Section 4.1):
    pins Hbar and the convolution P = psi * Hbar together."""
    rng = np.random.default_rng(5)
    n, d = 60, 4
    q = rng.uniform(0, 0.05, (n, d, d))
    q[0] = 0
    ps = orc.psi(q)
    P = orc.transition(ps, q)
    assert np.max(np.abs(P.sum(axis=2) - 1.0)) <= 1e-12
    assert np.array_equal(P[0], np.eye(d))


def test_renewal_equation_and_transition_equation(orc):
    """psi = e0 + q*psi and P = Hbar + q*P (eqs. renewal-sequence and
    transition-discrete) hold for the oracle's outputs."""
    k = si.weibull_kernel(4, 120, 11)
    q = k.q.numpy()
    ps = orc.psi(q)
    E = np.zeros_like(ps)
    E[0] = np.eye(4)
    assert np.max(np.abs(ps - (E + orc.conv(q, ps)))) <= 1e-14
    P = orc.transition(ps, q)
    H = np.zeros_like(ps)
    hb = orc.hbar(q)
    for t in range(q.shape[0]):
        H[t] = np.diag(hb[t])
    assert np.max(np.abs(P - (H + orc.conv(q, P)))) <= 1e-13


def test_finite_horizon_exactness(orc):
    """Proposition 2.3: the first n' coefficients depend only on q(0..n'-1)."""
    k = si.weibull_kernel(3, 100, 12)
    q = k.q.numpy()
    full = orc.psi(q)
    pre = orc.psi(q[:40])
    assert np.array_equal(full[:40], pre)
    q2 = q.copy()
    q2[40:] *= 0.5
    assert np.array_equal(orc.psi(q2)[:40], full[:40])


def test_nonnegative_and_substochastic(orc):
    """psi >= 0, and for k >= 1 at most one renewal happens at time k, so each
    row of psi(k) sums to <= 1; P is a stochastic matrix."""
    for fam in ("weibull", "lognormal"):
        k = si.family_kernel(fam, 5, 200, 21)
        q = k.q.numpy()
        ps = orc.psi(q)
        assert ps.min() >= -1e-15
        assert ps[1:].sum(axis=2).max() <= 1 + 1e-13
        P = orc.transition(ps, q)
        assert P.min() >= -1e-15


def test_transpose_symmetry(orc):
    """(e0 - q^T)^-1 = ((e0 - q)^-1)^T coefficientwise: catches a swapped
    product order in any one-sided formula."""
    k = si.weibull_kernel(5, 90, 13)
    q = k.q.numpy()
    a = orc.psi(q)
    b = orc.psi(np.ascontiguousarray(q.transpose(0, 2, 1)))
    assert np.max(np.abs(a - b.transpose(0, 2, 1))) <= 1e-14


def test_residual_bound_proposition(orc):
    """Proposition 2.6 on a perturbed inverse: ||psi - X||_{1,N} <=
    ||rho||/(1-||rho||) ||X||_{1,N} whenever ||rho||_{1,N} < 1."""
    k = si.weibull_kernel(3, 64, 14)
    q = k.q.numpy()
    ps = orc.psi(q)
    rng = np.random.default_rng(0)
    X = ps + 1e-6 * rng.standard_normal(ps.shape)
    A = orc.e0_minus(q)
    rL, rR = orc.residuals(A, X)
    err = orc.norm_1N(ps - X)
    for r in (rL, rR):
        nr = orc.norm_1N(r)
        assert nr < 1
        assert err <= nr / (1 - nr) * orc.norm_1N(X) * (1 + 1e-12)


def test_paper_first_entrance_worked_example(orc):
    """Section 5.1 first-restoration example (Poisson 8, 5, 10, 7; D = {1},
    C = {2, 3}, alpha_C = (1, 0), N = 128).  From the degraded state the chain
    either returns directly (prob 1/5, 1 + Poisson(5) steps) or goes through
    shutdown (prob 4/5, 2 + Poisson(10) + Poisson(7) = 2 + Poisson(17) steps),
    so the mass has a closed form; the paper reports that the cumulative
    probability at the last time is one to the displayed precision."""
    from scipy.stats import poisson
    n = 128
    k = si.paper_three_state_poisson(n)
    q = k.q.numpy()
    inD = np.array([1, 0, 0])
    alpha = np.array([0.0, 1.0, 0.0])
    ga, F = orc.first_entrance(q, inD, alpha)
    t = np.arange(n)
    ref = 0.2 * np.where(t >= 1, poisson.pmf(t - 1, 5.0), 0) + 0.8 * np.where(t >= 2, poisson.pmf(t - 2, 17.0), 0)
    assert np.max(np.abs(ga - ref)) <= 1e-15
    assert abs(F[-1] - 1.0) <= 1e-14


def test_adjoint_matches_forward_mode(orc):
    """<qbar, dq> = <psibar, dpsi>: the adjoint (linearised resolvent identity,
    Prop. 2.5) against forward mode on the renewal equation psi = e0 + q*psi."""
    rng = np.random.default_rng(6)
    k = si.weibull_kernel(4, 48, 15)
    q = k.q.numpy()
    ps = orc.psi(q)
    pb = rng.standard_normal(ps.shape)
    qb = orc.adjoint(ps, pb)
    for _ in range(3):
        dq = rng.standard_normal(q.shape)
        dq[0] = 0
        dps = orc.forward_mode(q, ps, dq)
        lhs = np.sum(qb[1:] * dq[1:])
        rhs = np.sum(pb * dps)
        assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))


def test_forward_mode_matches_central_difference(orc):
    """Forward mode against a central finite difference of the oracle itself."""
    rng = np.random.default_rng(7)
    k = si.weibull_kernel(3, 40, 16)
    q = k.q.numpy()
    ps = orc.psi(q)
    dq = rng.standard_normal(q.shape)
    dq[0] = 0
    h = 1e-6
    fd = (orc.psi(q + h * dq) - orc.psi(q - h * dq)) / (2 * h)
    dps = orc.forward_mode(q, ps, dq)
    assert np.max(np.abs(fd - dps)) <= 1e-7 * max(1.0, np.max(np.abs(dps)))


def test_row_recursion_matches_full(orc):
    rng = np.random.default_rng(8)
    A = _rand_series(rng, 30, 5)
    al = rng.standard_normal(5)
    r = orc.series_inverse_row(A, al)
    X = orc.series_inverse_left(A)
    assert np.max(np.abs(r - np.einsum("i,kij->kj", al, X))) <= 1e-13


def test_column_subset_matches_full(orc):
    rng = np.random.default_rng(9)
    A = _rand_series(rng, 30, 6)
    X = orc.series_inverse_left(A)
    cols = [0, 3, 5]
    Xc = orc.series_inverse_left(A, cols)
    assert np.array_equal(Xc, X[:, :, cols])


def test_paper_residual_orders(orc):
    """Horizon-scaling model at N = 128: the recursion's own residuals are far
    below the FFT-Newton residuals the paper reports (5.71e-15 / 5.91e-15)."""
    k = si.paper_three_state_gamma(128)
    q = k.q.numpy()
    ps = orc.psi(q)
    rL, rR = orc.residuals(orc.e0_minus(q), ps)
    assert orc.norm_1N(rL) < 5.71e-15 * 10
    assert orc.norm_1N(rR) < 5.91e-15 * 10



UP, DOWN = [0, 1, 2], [3]
ALPHA = np.array([1.0, 0.0, 0.0, 0.0])


def _exact(G, t):
    """Exact Markov availability alpha exp(G t) 1_U and reliability
    alpha_U exp(G_UU t) 1_U (Section 5.2), by scipy's matrix exponential."""
    from scipy.linalg import expm
    P = np.stack([expm(G * tm) for tm in t])
    R = np.array([expm(G[np.ix_(UP, UP)] * tm)[0].sum() for tm in t])
    return P, P[:, 0, UP].sum(1), R


def _mean_value(orc, Q, Hb, n):
    """Mean-value approximation (Section 4.2) of P, availability and
    reliability on t_0 .. t_{n-1}, from the kernel Q sampled on t_0 .. t_n and
    the survival Hb:
    K_h = (e0 - Qbar_h)^-1 * [L_h - 1/2 Delta^+Q_h * (L_h(0) e0)], with
    L = Hbar for P and L = Q_UD (first entrance into D = {3}) for reliability,
    through oracle.mre_mean_value (general-A(0) inverse, Qbar_h(0) != 0)."""
    s = Q.shape[1]
    P = orc.mre_mean_value(Q[:n + 1], Hb[:n])
    GD = orc.mre_mean_value(Q[:n + 1][:, UP][:, :, UP], Q[:n][:, UP][:, :, DOWN])
    return P, P[:, 0, UP].sum(1), 1.0 - GD[:, 0, 0]


def _process(orc, Q, n):
    """Process discretization (Section 4.2): the discrete renewal sequence of
    q = Delta Q_h (q(0) = 0) and the oracle's availability and reliability
    (Section 4.1) on t_0 .. t_{n-1}."""
    q = np.zeros((n,) + Q.shape[1:])
    q[1:] = Q[1:n] - Q[:n - 1]
    up = np.array([1, 1, 1, 0])
    return orc.availability(q, up, ALPHA), orc.reliability(q, up, ALPHA)


def test_paper_exponential_convergence_table(orc):
    """The paper's fixed-horizon refinement table (Section 5.2): the
    mean-value scheme for the four-state exponential model, run through the
    oracle's general-A(0) inverse and rectangular convolutions, reproduces
    every printed error to its five significant digits and every printed
    order to three decimals (fixture golden/exponential_convergence.txt).
    The embedded matrix derived from the generator is the printed one."""
    fx = pf.read_blocks("exponential_convergence.txt")
    G, T = pf.generator(fx), float(fx["horizon"])
    lam = [-Fraction(str(G[i, i])) for i in range(4)]
    derived = [[Fraction(0) if i == j else Fraction(str(G[i, j])) / lam[i] for j in range(4)] for i in range(4)]
    assert derived == pf.embedded(fx)
    prev = None
    for row in fx["table"]:
        h = float(row[0])
        n = int(np.floor(T / h + 1e-9)) + 1
        P, A, R = _mean_value(orc, *si.exponential_semi_markov(G, h, n + 1), n)
        Pex, Aex, Rex = _exact(G, h * np.arange(n))
        errs = (np.max(np.linalg.norm(P - Pex, axis=(1, 2))), np.max(np.abs(R - Rex)), np.max(np.abs(A - Aex)))
        for c, e in enumerate(errs):
            assert pf.same_digits(e, row[1 + 2 * c]), (h, c, e, row[1 + 2 * c])
            if prev is None:
                assert row[2 + 2 * c] == "-"
            else:
                assert pf.same_digits(np.log2(prev[c] / e), row[2 + 2 * c], 3), (h, c, row[2 + 2 * c])
        prev = errs


def test_paper_exponential_long_horizon(orc):
    """The paper's long-horizon errors for the same model (Section 5.2,
    N = 2^15, h = 0.005; fixture golden/exponential_figure.txt), to the
    printed three digits.  The process discretization is the discrete path
    itself: the renewal sequence of q = Delta Q_h (q(0) = 0) with the oracle's
    availability and reliability functions (Section 4.1)."""
    fx = pf.read_blocks("exponential_figure.txt")
    G, h, n = pf.generator(fx), float(fx["h"]), int(fx["N"])
    printed = {r[0]: r[1:] for r in fx["errors"]}
    _, Aex, Rex = _exact(G, h * np.arange(n))
    Q, Hb = si.exponential_semi_markov(G, h, n + 1)
    A, R = _process(orc, Q, n)
    for e, v in zip((np.max(np.abs(A - Aex)), np.max(np.abs(R - Rex))), printed["process"]):
        assert pf.same_digits(e, v), (e, v)
    _, A, R = _mean_value(orc, Q, Hb, n)
    for e, v in zip((np.max(np.abs(A - Aex)), np.max(np.abs(R - Rex))), printed["mean_value"]):
        assert pf.same_digits(e, v), (e, v)


def test_paper_lognormal_scheme_difference(orc):
    """The heavy-tailed lognormal model of Section 5.2 (parameters from the
    appendix; fixture golden/lognormal_figure.txt): on the N = 2^15,
    h = 0.005 grid the mean-value approximation and the process
    discretization differ by at most the printed amounts in availability and
    reliability, to the printed three digits."""
    fx = pf.read_blocks("lognormal_figure.txt")
    pemb = pf.embedded_matrix(fx)
    mu, sigma = pf.lognormal_params(fx, 4)
    h, n = float(fx["h"]), int(fx["N"])
    printed = dict(fx["differences"])
    Q, Hb = si.lognormal_semi_markov(pemb, mu, sigma, h, n + 1)
    A_pd, R_pd = _process(orc, Q, n)
    _, A_mv, R_mv = _mean_value(orc, Q, Hb, n)
    assert pf.same_digits(np.max(np.abs(A_mv - A_pd)), printed["max_dA"])
    assert pf.same_digits(np.max(np.abs(R_mv - R_pd)), printed["max_dR"])


def test_geometric_helpers_match_the_pinned_recursion(orc):
    """The closed-form helpers used as checkers at full size (geometric_psi,
    geometric_P) against the left recursion and P = psi*Hbar, which the path
    enumeration and the inline closed form above pin.  A helper with a wrong
    power (M^k instead of M^(k-1)), a missing -diag(a) or a transposed M fails."""
    d, n = 5, 60
    k = si.geometric_kernel(d, n, 12)
    q = k.q.numpy()
    M, a = k.params["M"], k.params["a"]
    ks = np.arange(n)
    ps = orc.psi(q)
    assert np.max(np.abs(orc.geometric_psi(M, a, ks) - ps)) <= 1e-14
    assert np.max(np.abs(orc.geometric_P(M, ks) - orc.transition(ps, q))) <= 1e-13
    # Sampled, out-of-order coefficient lists return the same values.
    sub = np.array([37, 0, 5, 59, 1])
    assert np.max(np.abs(orc.geometric_psi(M, a, sub) - ps[sub])) <= 1e-14
    # The planted mistakes named above are all visible at this size.
    wrong = [np.linalg.matrix_power(M, t) @ (M - np.diag(a)) for t in range(1, 8)]
    assert np.max(np.abs(np.array(wrong) - ps[1:8])) > 1e-3
    wrong = [np.linalg.matrix_power(M, t - 1) @ M for t in range(1, 8)]
    assert np.max(np.abs(np.array(wrong) - ps[1:8])) > 1e-3
    wrong = [np.linalg.matrix_power(M.T, t - 1) @ (M.T - np.diag(a)) for t in range(1, 8)]
    assert np.max(np.abs(np.array(wrong) - ps[1:8])) > 1e-3


def test_residuals_fft_matches_direct_residuals(orc):
    """The numpy-FFT residual checker (residuals_fft) against the direct
    residual sequences e0 - A*X and e0 - X*A of eq. (convolution) on a
    perturbed inverse, where left and right residuals differ (matrix products
    do not commute), so a swapped operand order or a dropped e0 fails."""
    rng = np.random.default_rng(21)
    d, n = 4, 50
    q = si.weibull_kernel(d, n, 21).q.numpy()
    X = orc.psi(q) + 1e-6 * rng.standard_normal((n, d, d))
    RL, RR = orc.residuals(orc.e0_minus(q), X)
    rl, rr, ml, mr_ = orc.residuals_fft(q, X, row_block=3)
    fro = lambda R: float(np.sum(np.linalg.norm(R, axis=(1, 2))))
    assert abs(rl - fro(RL)) <= 1e-12 * fro(RL)
    assert abs(rr - fro(RR)) <= 1e-12 * fro(RR)
    assert abs(ml - np.max(np.abs(RL))) <= 1e-15 and abs(mr_ - np.max(np.abs(RR))) <= 1e-15
    assert abs(rl - rr) > 1e-3 * rl
    # The exact inverse has residuals at rounding level.
    rl0, rr0, ml0, mr0 = orc.residuals_fft(q, orc.psi(q))
    assert ml0 <= 1e-15 and mr0 <= 1e-15


def test_sampled_residual_closed_form(orc):
    """residual_at: e0 - A*X at chosen coefficients by the direct sum.  Pins:
    the exact inverse leaves rounding only; a perturbation eps at X(k0) alone
    gives rho(k) = -A(k - k0) eps for k >= k0 and leaves rho(k < k0) unchanged;
    the values at every k equal the direct residual sequence."""
    rng = np.random.default_rng(22)
    d, n = 3, 40
    A = _rand_series(rng, n, d)
    X = orc.series_inverse_left(A)
    ks = np.array([0, 1, 7, 20, 39])
    assert np.max(np.abs(orc.residual_at(A, X, ks))) <= 1e-14
    eps = rng.standard_normal((d, d)) * 1e-3
    k0 = 7
    Xp = X.copy()
    Xp[k0] += eps
    got = orc.residual_at(A, Xp, ks)
    for s, k in enumerate(ks):
        ref = -A[k - k0] @ eps if k >= k0 else np.zeros((d, d))
        assert np.max(np.abs(got[s] - ref)) <= 1e-14
    RL, _ = orc.residuals(A, Xp)
    assert np.max(np.abs(orc.residual_at(A, Xp, np.arange(n)) - RL)) <= 1e-15
    # With e0_minus the first argument is q and A = e0 - q.
    q = si.weibull_kernel(d, n, 23).q.numpy()
    ps = orc.psi(q) + 1e-5
    assert np.max(np.abs(orc.residual_at(q, ps, ks, e0_minus=True)
                         - orc.residual_at(orc.e0_minus(q), ps, ks))) <= 1e-16
    with pytest.raises(ValueError):
        orc.residual_at(A, X, [n])


def test_recursion_sums_do_not_depend_on_the_thread_count(orc):
    """The recursions cut their inner sums into a fixed number of chunks, so
    the oracle gives the same bits whatever OpenMP team it runs on."""
    import subprocess
    import sys
    code = ("import hashlib, numpy as np, smk_inputs as si, oracle; "
            "q = si.weibull_kernel(6, 1500, 24).q.numpy(); "
            "x = oracle.psi(q); r = oracle.series_inverse_row(oracle.e0_minus(q), np.eye(6)[1]); "
            "print(hashlib.sha256(x.tobytes() + r.tobytes()).hexdigest())")
    import os
    outs = []
    for th in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=th)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                   cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                   check=True).stdout.strip())
    assert outs[0] == outs[1]


def test_mean_value_scheme_planted_mistakes(orc):
    """mre_mean_value is pinned by the printed convergence table above; these
    are the plausible slips that table rules out, checked to move the h = 0.1
    errors by far more than its five digits: A(0) taken as I, the Delta+
    correction dropped, and Delta Q in place of Qbar (the process scheme)."""
    fx = pf.read_blocks("exponential_convergence.txt")
    G, T = pf.generator(fx), float(fx["horizon"])
    h = 0.1
    n = int(np.floor(T / h + 1e-9)) + 1
    Q, Hb = si.exponential_semi_markov(G, h, n + 1)
    Pex, _, _ = _exact(G, h * np.arange(n))
    good = np.max(np.linalg.norm(orc.mre_mean_value(Q, Hb[:n]) - Pex, axis=(1, 2)))
    dQ = np.zeros_like(Q)
    dQ[1:] = Q[1:] - Q[:-1]
    Qbar = 0.5 * (dQ[:n] + dQ[1:n + 1])
    A = -Qbar
    A[0] = np.eye(4)                                           # slip 1: A(0) = I
    slip1 = orc.conv(orc.series_inverse_left(A), Hb[:n] - 0.5 * np.matmul(dQ[1:n + 1], Hb[0]))
    A = -Qbar
    A[0] += np.eye(4)
    slip2 = orc.conv(orc.series_inverse_left(A), Hb[:n])       # slip 2: no Delta+ correction
    A = -dQ[:n]
    A[0] += np.eye(4)
    slip3 = orc.conv(orc.series_inverse_left(A), Hb[:n])       # slip 3: the process scheme
    for bad in (slip1, slip2, slip3):
        e = np.max(np.linalg.norm(bad - Pex, axis=(1, 2)))
        assert e > 3 * good, (e, good)


def test_renewal_visits_closed_forms(orc):
    """Renewal visits N_B(k) = alpha sum_{l<=k} psi(l) I_B 1 (eq.
    (renewal-visits)): for d = 1 geometric sojourns every step renews with
    probability 1 - a, so N(k) = 1 + k (1 - a); for the Markov case
    N_B(k) = alpha [I_B 1 + sum_{l=1..k} M^(l-1) (M - diag a) 1_B]; summed over
    a partition of E the visits add up."""
    a, n = 0.7, 50
    q = np.zeros((n, 1, 1))
    q[1:, 0, 0] = (1 - a) * a ** np.arange(n - 1)
    N = orc.renewal_visits(q, [1], [1.0])
    assert np.max(np.abs(N - (1 + np.arange(n) * (1 - a)))) <= 1e-13
    d, n = 5, 60
    k = si.geometric_kernel(d, n, 14)
    M, av = k.params["M"], k.params["a"]
    alpha = np.array([0.2, 0.0, 0.5, 0.3, 0.0])
    inB = np.array([1, 0, 0, 1, 1])
    ref = np.empty(n)
    acc = alpha @ inB
    Mk = np.eye(d)
    ref[0] = acc
    for t in range(1, n):
        acc += alpha @ Mk @ (M - np.diag(av)) @ inB
        ref[t] = acc
        Mk = Mk @ M
    got = orc.renewal_visits(k.q.numpy(), inB, alpha)
    assert np.max(np.abs(got - ref)) <= 1e-12
    other = orc.renewal_visits(k.q.numpy(), 1 - inB, alpha)
    every = orc.renewal_visits(k.q.numpy(), np.ones(d), alpha)
    assert np.max(np.abs(got + other - every)) <= 1e-12


def test_monte_carlo_oracle_markov_closed_form(orc):
    """The oracle's pathwise Monte Carlo (the Section 5.2 validation method)
    on exponential sojourns, where the process is the Markov chain of the
    exponential benchmark's generator: availability alpha exp(G t) 1_U and
    reliability alpha_U exp(G_UU t) 1 hold within 5.5 binomial standard
    deviations at every grid point.  A sampler that picks the wrong next
    state, uses the wrong rate or marks the wrong grid cells fails by far more."""
    from scipy.linalg import expm
    G = pf.generator(pf.read_blocks("exponential_convergence.txt"))
    lam = -np.diag(G)
    P = G / lam[:, None]
    np.fill_diagonal(P, 0.0)
    rate = np.repeat(lam[:, None], 4, axis=1)
    h, n, M = 0.05, 400, 200000
    A, R = orc.semi_markov_mc(P, rate, np.ones((4, 4)), [1, 1, 1, 0], h, n, M, 11, family="exponential")
    t = h * np.arange(n)
    Aex = np.array([expm(G * x)[0, :3].sum() for x in t])
    Rex = np.array([expm(G[:3, :3] * x)[0].sum() for x in t])
    for est, ex in ((A, Aex), (R, Rex)):
        sd = np.sqrt(np.maximum(ex * (1 - ex), 1e-6) / M)
        assert np.max(np.abs(est - ex) / sd) <= 5.5
    # planted: the same simulation with the rates swapped between states is far off
    A2, _ = orc.semi_markov_mc(P, rate[::-1].copy(), np.ones((4, 4)), [1, 1, 1, 0], h, n, M, 11, family="exponential")
    assert np.max(np.abs(A2 - Aex)) > 20 * np.max(np.sqrt(Aex * (1 - Aex) / M))


def test_monte_carlo_oracle_lognormal_sojourn_law(orc):
    """The lognormal sampler: a two-state alternating process whose first
    sojourn is lognormal(mu, sigma) has R(t) = P(T > t) = 1 - Phi((ln t - mu)/
    sigma) for the down state entered at the first jump; the estimate holds
    within 5.5 standard deviations.  The stream is deterministic: the same
    seed repeats bit for bit, another seed differs."""
    from scipy.stats import norm
    P = np.array([[0.0, 1.0], [1.0, 0.0]])
    mu, sg = np.array([[0.0, 1.2], [0.0, 0.0]]), np.array([[1.0, 0.7], [1.0, 1.0]])
    h, n, M = 0.05, 300, 200000
    A, R, tau, jumps = orc.semi_markov_mc(P, mu, sg, [1, 0], h, n, M, 12, per_path=True)
    t = h * np.arange(n)
    Rex = np.where(t > 0, 1.0 - norm.cdf((np.log(np.maximum(t, 1e-300)) - 1.2) / 0.7), 1.0)
    sd = np.sqrt(np.maximum(Rex * (1 - Rex), 1e-6) / M)
    assert np.max(np.abs(R - Rex) / sd) <= 5.5
    again = orc.semi_markov_mc(P, mu, sg, [1, 0], h, n, M, 12, per_path=True)
    assert np.array_equal(again[2], tau) and np.array_equal(again[3], jumps)
    other = orc.semi_markov_mc(P, mu, sg, [1, 0], h, n, M, 13, per_path=True)
    assert not np.array_equal(other[2], tau)


def test_philox_stream_statistics(orc):
    """Philox4x32-10 blocks: words are uniform on 32 bits (mean and a 64-bin
    chi-square over 2^14 blocks) and one flipped counter bit changes about
    half of the 128 output bits."""
    words = np.array([orc.philox4x32_10([k, 0, 5, 0], [123, 456]) for k in range(1 << 14)]).ravel()
    u = words / 2.0 ** 32
    assert abs(u.mean() - 0.5) <= 5 * np.sqrt(1 / 12 / u.size)
    counts = np.bincount((words >> 26).astype(np.int64), minlength=64)
    chi2 = float(np.sum((counts - u.size / 64) ** 2 / (u.size / 64)))
    assert chi2 <= 130                      # 63 degrees of freedom: far beyond the 1e-6 quantile
    a = orc.philox4x32_10([1, 2, 3, 4], [5, 6])
    flips = []
    for bit in range(32):
        b = orc.philox4x32_10([1 ^ (1 << bit), 2, 3, 4], [5, 6])
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert 48 <= np.mean(flips) <= 80
