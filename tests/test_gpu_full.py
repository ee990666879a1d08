"""Full-size GPU checks of the named workloads, in the launch configuration
bench.py times (one call of the C-ABI per inversion, default stream).

At these sizes the quadratic oracle cannot produce every output, so each
test combines:
  * oracle values on a prefix (exact sub-problem by finite-horizon exactness,
    Proposition 2.3): the full matrix on a short prefix and sampled columns
    or rows on a longer one;
  * closed forms at any horizon (the Markov case, geometric sojourns);
  * identities that hold at any size (row sums of P equal one, residuals
    e0 - A*psi computed with numpy's own FFT, independent of the GPU code).
"""
import math

import numpy as np
import pytest
import torch

import smk_inputs as si

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


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def test_c2_fp64_full_size(mr, orc):
    """d = 16, n = 65536, Weibull (seed 1), FP64: max-abs <= 1e-12."""
    d, n = 16, 65536
    print("[c2] generating", flush=True)
    k = si.weibull_kernel(d, n, si.CONFIG_SEEDS["c2"], device="cuda")
    psi = mr.psi_inverse(k.q, "fp64", check=True)
    P = mr.transition(psi, k.q)
    qh = k.q[:2048].cpu().numpy()
    ref = orc.psi(qh)
    assert _maxerr(_np(psi[:2048]), ref) <= 1e-12
    print("[c2] prefix column", flush=True)
    npre = 8192
    col = orc.psi(k.q[:npre].cpu().numpy(), cols=[5])
    assert _maxerr(_np(psi[:npre, :, 5:6]), col) <= 1e-12
    # Exact identity at every k: rows of P sum to one.
    assert float((P.sum(dim=2) - 1).abs().max()) <= 1e-12
    # Residuals over the whole horizon with numpy's FFT (Proposition 2.6 inputs).
    print("[c2] residuals", flush=True)
    rl, rr, ml, mrr = orc.residuals_fft(k.q.cpu().numpy(), _np(psi))
    print(f"[c2] residual sums {rl:.3e} {rr:.3e} max {ml:.3e} {mrr:.3e}", flush=True)
    assert ml <= 1e-13 and mrr <= 1e-13


def test_c2_markov_closed_form_full_size(mr, orc):
    """Geometric sojourns (seed 2), d = 16, n = 65536: psi(k) = M^(k-1)(M - diag a)
    and P(k) = M^k at sampled k across the whole horizon."""
    d, n = 16, 65536
    k = si.geometric_kernel(d, n, si.CONFIG_SEEDS["c2_geom"], device="cuda")
    psi = mr.psi_inverse(k.q, "fp64", check=True)
    P = mr.transition(psi, k.q)
    ks = np.unique(np.concatenate([np.arange(0, 40), np.linspace(40, n - 1, 60).astype(int)]))
    kt = torch.as_tensor(ks, device="cuda")
    assert _maxerr(_np(psi[kt]), orc.geometric_psi(k.params["M"], k.params["a"], ks)) <= 1e-12
    assert _maxerr(_np(P[kt]), orc.geometric_P(k.params["M"], ks)) <= 1e-12


def test_c3_markov_closed_form_mixed(mr, orc):
    """Mixed form on the Markov case at d = 64, n = 262144."""
    d, n = 64, 262144
    k = si.geometric_kernel(d, n, 33, device="cuda")
    psim = mr.psi_inverse(k.q, "mixed", check=True)
    ks = np.unique(np.linspace(0, n - 1, 40).astype(int))
    kt = torch.as_tensor(ks, device="cuda")
    assert _maxerr(_np(psim[kt]), orc.geometric_psi(k.params["M"], k.params["a"], ks)) <= 1e-10


def _c5_loss(mr, q, up, alpha, target):
    """sum_k A(k) + F_{target}(n-1) through the library's autograd Functions."""
    d = q.shape[1]
    psi = mr.PsiInverse.apply(q)
    P = mr.Transition.apply(psi, q)
    A = mr.Contract.apply(P, alpha, up)
    C = [i for i in range(d) if i != target]
    qCC = mr.GatherBlock.apply(q, C, C)
    qCD = mr.GatherBlock.apply(q, C, [target])
    g = mr.RenewalApply.apply(mr.PsiInverse.apply(qCC), qCD)
    aC = torch.zeros(d - 1, dtype=torch.float64)
    aC[0] = 1.0
    F = mr.Contract.apply(g, aC, torch.ones(1, dtype=torch.float64), True)
    return A.sum() + F[-1]


def test_c5_gradient_chain_matches_oracle_forward_mode(mr, orc):
    """The GPU gradient of the full loss with respect to q, contracted with a
    random direction dq, against the oracle's forward-mode derivative of the
    same chain (dpsi = dq*psi + q*dpsi, dP = dpsi*Hbar + psi*dHbar, ...)."""
    d, n, target = 6, 200, 5
    k = si.weibull_kernel(d, n, 55)
    up = torch.tensor([1.0] * 3 + [0.0] * 3, dtype=torch.float64)
    alpha = torch.zeros(d, dtype=torch.float64)
    alpha[0] = 1.0
    q = k.q.cuda().requires_grad_(True)
    _c5_loss(mr, q, up, alpha, target).backward()
    g = _np(q.grad)
    rng = np.random.default_rng(5)
    qn = k.q.numpy()
    for _ in range(2):
        dq = rng.standard_normal(qn.shape)
        dq[0] = 0
        psi = orc.psi(qn)
        dpsi = orc.forward_mode(qn, psi, dq)
        hb = orc.hbar(qn)
        dhb = -np.cumsum(dq.sum(axis=2), axis=0)
        dhb[0] = 0.0
        H = np.zeros((n, d, d))
        dH = np.zeros((n, d, d))
        for t in range(n):
            H[t] = np.diag(hb[t])
            dH[t] = np.diag(dhb[t])
        dP = orc.conv(dpsi, H) + orc.conv(psi, dH)
        dA = np.einsum("i,kij,j->", alpha.numpy(), dP, up.numpy())
        C = [i for i in range(d) if i != target]
        qCC = np.ascontiguousarray(qn[:, C][:, :, C])
        qCD = np.ascontiguousarray(qn[:, C][:, :, [target]])
        dCC = np.ascontiguousarray(dq[:, C][:, :, C])
        dCD = np.ascontiguousarray(dq[:, C][:, :, [target]])
        psiC = orc.psi(qCC)
        dpsiC = orc.forward_mode(qCC, psiC, dCC)
        dg = orc.conv(dpsiC, qCD) + orc.conv(psiC, dCD)
        dF = dg[:, 0, 0].sum()
        ref = dA + dF
        got = float(np.sum(g * dq))
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_c5_psi_against_oracle(mr, orc, form):
    """The inverse under the gradient workload, d = 32, n = 65536, Weibull
    (seed 5): psi against the oracle on the prefix k < 4096 (finite-horizon
    exactness), and the oracle's direct left residual e0 - A*psi at sampled
    coefficients up to n - 1."""
    d, n = 32, 65536
    k = si.weibull_kernel(d, n, si.CONFIG_SEEDS["c5"], device="cuda")
    psi = mr.psi_inverse(k.q, form, check=True)
    qh = _np(k.q)
    npre = 4096
    ref = orc.psi(qh[:npre])
    tol = 1e-12 if form == "fp64" else 1e-10
    e = _maxerr(_np(psi[:npre]), ref)
    ks = np.array([1, 3000, 9000, 20000, 33000, 47000, n - 2, n - 1])
    rho = float(np.max(np.abs(orc.residual_at(qh, _np(psi), ks, e0_minus=True))))
    print(f"[c5 {form}] prefix {npre}: {e:.3e}; residual at {len(ks)} coefficients: {rho:.3e}", flush=True)
    assert e <= tol and rho <= tol


def test_c5_full_size_gradients_vs_central_differences(mr):
    """d = 32, n = 65536, Weibull (seed 5).  Loss = sum_k A(k) (U = first 16
    states) + first-entrance probability into state d-1 at n-1.  Gradients with
    respect to every Weibull shape, scale and jump logit (3 d (d-1) = 2976 live
    parameters) through the adjoint kernels, checked along random directions
    against central differences with h = 1e-6 in FP64."""
    d, n, target = 32, 65536, 31
    shape, scale, logits = si.weibull_params(d, si.CONFIG_SEEDS["c5"], device="cuda")
    up = torch.tensor([1.0] * 16 + [0.0] * 16, dtype=torch.float64)
    alpha = torch.zeros(d, dtype=torch.float64)
    alpha[0] = 1.0
    params = [t.clone().requires_grad_(True) for t in (shape, scale, logits)]
    loss = _c5_loss(mr, si.weibull_kernel_from_params(*params, n), up, alpha, target)
    loss.backward()
    grads = [p.grad.detach() for p in params]
    off = ~torch.eye(d, dtype=torch.bool, device="cuda")
    for g in grads:
        assert torch.isfinite(g).all()
        assert float(g[~off].abs().max()) == 0.0          # diagonal entries do not enter q
    assert int(sum(int((g[off] != 0).sum()) for g in grads)) == 3 * d * (d - 1)
    gen = torch.Generator(device="cpu").manual_seed(0)
    h = 1e-6
    for trial in range(3):
        dirs = [torch.randn(d, d, generator=gen, dtype=torch.float64).cuda() * off for _ in range(3)]
        with torch.no_grad():
            lp = _c5_loss(mr, si.weibull_kernel_from_params(*[p + h * v for p, v in zip(params, dirs)], n),
                          up, alpha, target)
            lm = _c5_loss(mr, si.weibull_kernel_from_params(*[p - h * v for p, v in zip(params, dirs)], n),
                          up, alpha, target)
        fd = float((lp - lm) / (2 * h))
        an = float(sum((g * v).sum() for g, v in zip(grads, dirs)))
        print(f"[c5] trial {trial}: adjoint {an:.10e} fd {fd:.10e} rel {abs(an - fd) / abs(an):.2e}", flush=True)
        assert abs(an - fd) <= 1e-5 * abs(an)


def test_c4_batched_uneven_workload(mr, orc):
    """512 problems, d uniform in 3..48, n log-uniform in [1024, 32768],
    Weibull or lognormal by coin flip (master seed 4), mixed form in one
    batched call.  32 sampled problems against the oracle on a prefix, 8 of
    them bitwise against the single-problem call, and for all 512 the
    invariants psi >= 0 and substochastic rows (k >= 1)."""
    work = si.batch_workload(si.CONFIG_SEEDS["c4"], 512)
    print("[c4] generating", flush=True)
    qs = [si.family_kernel(w["family"], w["d"], w["n"], w["seed"], device="cuda").q for w in work]
    print("[c4] batched inversion", flush=True)
    outs = mr.psi_inverse_batched(qs, "mixed")
    mr.sync_status()
    rng = np.random.default_rng(4)
    sample = rng.choice(len(work), 32, replace=False)
    for j, b in enumerate(sample):
        q, o = qs[b], outs[b]
        npre = 256 if work[b]["d"] > 32 else 512
        ref = orc.psi(q[:npre].cpu().numpy())
        assert _maxerr(_np(o[:npre]), ref) <= 1e-10, work[b]
        if j < 8:
            single = mr.psi_inverse(q, "mixed")
            torch.cuda.synchronize()
            assert torch.equal(single, o), work[b]
    for w, o in zip(work, outs):
        assert float(o.min()) >= -1e-12, w
        assert float(o[1:].sum(dim=2).max()) <= 1 + 1e-10, w



def _continuous_schemes(mr, orc, Q, Hb, n):
    """Both discretizations of Section 4.2 through the library, for a kernel Q
    sampled on t_0 .. t_n and its survival Hb; returns availability and
    reliability on t_0 .. t_{n-1} as {scheme: (A, R)}.
      * process: psi of q = Delta Q_h (FP64), P = psi*Hbar, availability, and
        reliability by first entrance (Section 4.1);
      * mean_value: mrinv_mre_solve, K_h = (e0 - Qbar_h)^-1 * [L_h - 1/2
        Delta^+Q_h * (L_h(0) e0)] (general-A(0) inverse, rectangular product).
    The process inverse and the mean-value P are checked against the oracle on
    a 2048-step prefix (an exact sub-problem, Proposition 2.3)."""
    up, U, D = [1, 1, 1, 0], [0, 1, 2], [3]
    alpha = [1.0, 0.0, 0.0, 0.0]
    dev = torch.device("cuda")
    dQ = np.zeros_like(Q)
    dQ[1:] = Q[1:] - Q[:-1]
    out = {}

    q = torch.from_numpy(np.ascontiguousarray(dQ[:n])).to(dev)
    psi = mr.psi_inverse(q, "fp64")
    assert _maxerr(_np(psi[:2048]), orc.psi(dQ[:2048])) <= 1e-12
    out["process"] = (_np(mr.availability(mr.transition(psi, q), up, alpha)), _np(mr.reliability(q, up, alpha)))

    # Mean-value scheme (Section 4.2, eq. (mre-solution)) by the library:
    # L = Hbar gives P; L = Q_UD on the up block gives the first entrance.
    Qg = torch.from_numpy(np.ascontiguousarray(Q[:n + 1])).to(dev)
    P = mr.mre_solve(Qg, torch.from_numpy(np.ascontiguousarray(Hb[:n])).to(dev))
    assert _maxerr(_np(P[:2048]), orc.mre_mean_value(Q[:2049], Hb[:2048])) <= 1e-12
    QU = torch.from_numpy(np.ascontiguousarray(Q[:n + 1][:, U][:, :, U])).to(dev)
    GD = mr.mre_solve(QU, torch.from_numpy(np.ascontiguousarray(Q[:n][:, U][:, :, D])).to(dev))
    out["mean_value"] = (_np(mr.availability(P, up, alpha)), 1.0 - _np(GD)[:, 0, 0])
    return out


def test_paper_exponential_long_horizon(mr, orc):
    """The four-state exponential model of Section 5.2 at N = 2^15, h = 0.005
    (fixture golden/exponential_figure.txt): through the library, each
    scheme's maximum availability and reliability error against the exact
    Markov solution (scipy's expm) rounds to the value the paper prints."""
    from scipy.linalg import expm

    import paper_fixtures as pf

    fx = pf.read_blocks("exponential_figure.txt")
    G, h, n = pf.generator(fx), float(fx["h"]), int(fx["N"])
    U = [0, 1, 2]
    t = h * np.arange(n)
    Aex = np.array([expm(G * tm)[0, U].sum() for tm in t])
    Rex = np.array([expm(G[np.ix_(U, U)] * tm)[0].sum() for tm in t])
    res = _continuous_schemes(mr, orc, *si.exponential_semi_markov(G, h, n + 1), n)
    for r in fx["errors"]:
        A, R = res[r[0]]
        for e, v in zip((_maxerr(A, Aex), _maxerr(R, Rex)), r[1:]):
            assert pf.same_digits(e, v), (r[0], e, v)


def test_paper_lognormal_scheme_difference(mr, orc):
    """The lognormal model of Section 5.2 (appendix parameters; fixture
    golden/lognormal_figure.txt) at N = 2^15, h = 0.005: through the library,
    the largest differences between the two schemes in availability and
    reliability round to the printed values."""
    import paper_fixtures as pf

    fx = pf.read_blocks("lognormal_figure.txt")
    mu, sigma = pf.lognormal_params(fx, 4)
    h, n = float(fx["h"]), int(fx["N"])
    printed = dict(fx["differences"])
    res = _continuous_schemes(mr, orc, *si.lognormal_semi_markov(pf.embedded_matrix(fx), mu, sigma, h, n + 1), n)
    (A_pd, R_pd), (A_mv, R_mv) = res["process"], res["mean_value"]
    assert pf.same_digits(_maxerr(A_mv, A_pd), printed["max_dA"])
    assert pf.same_digits(_maxerr(R_mv, R_pd), printed["max_dR"])
