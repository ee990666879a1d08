"""The continuous-time mean-value path (Section 4.2) and the remaining
Table 2 functionals (renewal visits, reward), through the C-ABI.

mrinv_mre_solve forms Qbar_h and the right-hand side of eq. (mre-solution)
on the GPU, inverts e0 - Qbar_h (general A(0)) and applies the inverse.  It is
checked element by element against oracle.mre_mean_value (which the paper's
printed convergence table pins on the CPU), and the paper's Section 5.2
numbers are reproduced through it: every error and order of the fixed-horizon
refinement table, and the long-horizon errors of the exponential benchmark.
"""
import numpy as np
import pytest
import torch

import paper_fixtures as pf
import smk_inputs as si
from tolerances import FP64_TOL, MIXED_TOL

pytestmark = pytest.mark.gpu

UP, DOWN = [0, 1, 2], [3]


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


def _lognormal_model(h, count):
    fx = pf.read_blocks("lognormal_figure.txt")
    mu, sigma = pf.lognormal_params(fx, 4)
    return si.lognormal_semi_markov(pf.embedded_matrix(fx), mu, sigma, h, count)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,r,model", [(1, 1, "exp"), (2, 4, "exp"), (37, 4, "logn"), (600, 1, "exp"),
                                       (3000, 4, "logn")])
def test_mre_solve_matches_oracle(mr, orc, precision, n, r, model):
    print(f"[mre] n={n} r={r} {model} {precision}", flush=True)
    if model == "exp":
        G = pf.generator(pf.read_blocks("exponential_convergence.txt"))
        Q, Hb = si.exponential_semi_markov(G, 0.05, n + 1)
    else:
        Q, Hb = _lognormal_model(0.05, n + 1)
    L = Hb[:n] if r == 4 else Q[:n][:, :, 3:4]
    got = _np(mr.mre_solve(_gpu(Q), _gpu(L), precision))
    ref = orc.mre_mean_value(Q, L)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    assert _maxerr(got, ref) <= tol
    mr.sync_status()


def test_paper_convergence_table_through_the_library(mr, orc):
    """Every error (15) and observed order (12) of the paper's fixed-horizon
    refinement table (Section 5.2; fixture golden/exponential_convergence.txt)
    from mrinv_mre_solve: P with L = Hbar, reliability from the first entrance
    into D = {3} with L = Q_UD on the up block, availability alpha P 1_U."""
    from scipy.linalg import expm
    fx = pf.read_blocks("exponential_convergence.txt")
    G, T = pf.generator(fx), float(fx["horizon"])
    alpha = np.eye(4)[0]
    prev = None
    for row in fx["table"]:
        h = float(row[0])
        n = int(np.floor(T / h + 1e-9)) + 1
        Q, Hb = si.exponential_semi_markov(G, h, n + 1)
        Qg = _gpu(Q)
        P = _np(mr.mre_solve(Qg, _gpu(Hb[:n])))
        GD = _np(mr.mre_solve(_gpu(Q[:, UP][:, :, UP]), _gpu(Q[:n][:, UP][:, :, DOWN])))
        A, R = P[:, 0, UP].sum(1), 1.0 - GD[:, 0, 0]
        t = h * np.arange(n)
        Pex = np.stack([expm(G * tm) for tm in t])
        Rex = np.array([expm(G[np.ix_(UP, UP)] * tm)[0].sum() for tm in t])
        errs = (np.max(np.linalg.norm(P - Pex, axis=(1, 2))), np.max(np.abs(R - Rex)),
                np.max(np.abs(A - Pex[:, 0, UP].sum(1))))
        print(f"[table] h={h}: {errs[0]:.4e} {errs[1]:.4e} {errs[2]:.4e}", flush=True)
        for c, e in enumerate(errs):
            assert pf.same_digits(e, row[1 + 2 * c]), (h, c, e, row[1 + 2 * c])
            if prev is not None:
                assert pf.same_digits(np.log2(prev[c] / e), row[2 + 2 * c], 3), (h, c, row[2 + 2 * c])
        prev = errs
        # the library's availability functional on the same P
        Ag = _np(mr.availability(_gpu(P), [1, 1, 1, 0], alpha))
        assert _maxerr(Ag, A) <= 1e-14


@pytest.mark.parametrize("d,n", [(1, 50), (5, 60), (7, 3000)])
def test_renewal_visits_match_oracle(mr, orc, d, n):
    if d == 1:
        a = 0.7
        q = np.zeros((n, 1, 1))
        q[1:, 0, 0] = (1 - a) * a ** np.arange(n - 1)
        inB, alpha = [1], [1.0]
    else:
        q = si.weibull_kernel(d, n, 200 + d).q.numpy()
        inB = [1, 0] * (d // 2) + [1] * (d % 2)
        alpha = np.full(d, 1.0 / d)
    psi = mr.psi_inverse(_gpu(q))
    N = _np(mr.renewal_visits(psi, inB, alpha))
    ref = orc.renewal_visits(q, inB, alpha)
    assert _maxerr(N, ref) <= 1e-12 * max(1.0, float(np.max(np.abs(ref))))
    if d == 1:
        assert _maxerr(N, 1 + np.arange(n) * 0.3) <= 1e-12


def test_reward_equation(mr, orc):
    """Reward-type equation V = r + q*V solved as V = psi * r (eq. (reward)) for
    a rectangular reward r in S_{d,3}: against the oracle's convolution of its
    own psi with r, and the defining equation V - q*V = r through the oracle."""
    d, n, c = 6, 700, 3
    q = si.lognormal_kernel(d, n, 210).q.numpy()
    rng = np.random.default_rng(211)
    r = rng.uniform(0.0, 1.0, (n, d, c))
    V = _np(mr.markov_renewal_apply(mr.psi_inverse(_gpu(q)), _gpu(r)))
    assert _maxerr(V, orc.conv(orc.psi(q), r)) <= 1e-12 * float(np.max(np.abs(V)))
    assert _maxerr(V - orc.conv(q, V), r) <= 1e-12 * float(np.max(np.abs(V)))
