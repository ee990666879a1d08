"""Pathwise Monte Carlo of the semi-Markov process on the GPU (Section 5.2's
validation of the lognormal model), through the C-ABI.

Both the library and the oracle implement Philox4x32-10 from its published
definition and the same sampling rules, so on one seed they simulate the same
trajectories: per trajectory the number of jumps is equal and the first
entrance time agrees to rounding (transcendental functions may differ in the
last bit between the two math libraries).  At the paper's size (10^6
trajectories) the pointwise 95% half-width reproduces the printed maximum,
the deterministic mean-value curves stay within it, and the RMS discrepancy
is at the Monte Carlo noise level, of the printed order of magnitude.
"""
import numpy as np
import pytest
import torch

import paper_fixtures as pf
import smk_inputs as si

pytestmark = pytest.mark.gpu

UP = np.array([1, 1, 1, 0], dtype=np.int32)


@pytest.fixture(scope="module")
def mr():
    import paper_2605_30379_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _model():
    fx = pf.read_blocks("lognormal_figure.txt")
    mu, sigma = pf.lognormal_params(fx, 4)
    return pf.embedded_matrix(fx), mu, sigma, float(fx["h"]), int(fx["N"])


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_mc_trajectories_match_the_oracle(mr, orc):
    P, mu, sigma, h, n = _model()
    M = 20000
    A, R, tau, jumps = mr.semi_markov_mc(P, mu, sigma, UP, h, n, M, 2026, per_path=True)
    oA, oR, otau, ojumps = orc.semi_markov_mc(P, mu, sigma, UP, h, n, M, 2026, per_path=True)
    tau, jumps = _np(tau), _np(jumps)
    print(f"[mc] jumps {jumps.mean():.2f} per path, entered D by t_max: {(tau >= 0).mean():.3f}", flush=True)
    assert np.array_equal(jumps, ojumps)
    assert np.array_equal(tau < 0, otau < 0)
    hit = tau >= 0
    assert np.max(np.abs(tau[hit] - otau[hit]) / otau[hit]) <= 1e-12
    # integer counts: equal except where a sojourn end lies within rounding of a grid point
    cnt = lambda x: np.rint(np.asarray(x) * M).astype(np.int64)
    dA, dR = np.abs(cnt(_np(A)) - cnt(oA)), np.abs(cnt(_np(R)) - cnt(oR))
    print(f"[mc] grid points with differing counts: A {(dA > 0).sum()}, R {(dR > 0).sum()}", flush=True)
    assert dA.max() <= 2 and dR.max() <= 2
    assert (dA > 0).sum() <= 5 and (dR > 0).sum() <= 5
    mr.sync_status()


def test_mc_is_deterministic_and_seeded(mr):
    P, mu, sigma, h, n = _model()
    a1, r1 = mr.semi_markov_mc(P, mu, sigma, UP, h, 4096, 50000, 7)
    a2, r2 = mr.semi_markov_mc(P, mu, sigma, UP, h, 4096, 50000, 7)
    a3, _ = mr.semi_markov_mc(P, mu, sigma, UP, h, 4096, 50000, 8)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(r1, r2)
    assert not torch.equal(a1, a3)


def test_paper_lognormal_monte_carlo_validation(mr):
    """10^6 trajectories on the paper's grid (N = 2^15, h = 0.005): the largest
    pointwise 95% half-width 1.96 sqrt(p(1-p)/M) rounds to the printed 9.80e-4;
    the mean-value approximation (mrinv_mre_solve) differs from the Monte Carlo
    curves by less than that half-width in availability and reliability, as
    the paper reports; and the RMS discrepancies are at the noise level of one
    Monte Carlo realization, of the order of the printed ones (another random
    stream than the paper's, so only their size is comparable)."""
    fxm = pf.read_blocks("lognormal_monte_carlo.txt")
    P, mu, sigma, h, n = _model()
    M = int(fxm["trajectories"])
    A, R = mr.semi_markov_mc(P, mu, sigma, UP, h, n, M, 20260621)
    A, R = _np(A), _np(R)
    hw = 1.96 * np.sqrt(np.maximum(A * (1 - A), R * (1 - R)) / M)
    print(f"[mc] max half-width {hw.max():.3e}", flush=True)
    assert pf.same_digits(float(hw.max()), fxm["max_half_width"])
    Q, Hb = si.lognormal_semi_markov(P, mu, sigma, h, n + 1)
    dev = torch.device("cuda")
    Pm = mr.mre_solve(torch.from_numpy(Q).to(dev), torch.from_numpy(np.ascontiguousarray(Hb[:n])).to(dev))
    U, D = [0, 1, 2], [3]
    GD = mr.mre_solve(torch.from_numpy(np.ascontiguousarray(Q[:, U][:, :, U])).to(dev),
                      torch.from_numpy(np.ascontiguousarray(Q[:n][:, U][:, :, D])).to(dev))
    Amv = _np(Pm)[:, 0, :3].sum(axis=1)
    Rmv = 1.0 - _np(GD)[:, 0, 0]
    dA, dR = np.abs(Amv - A), np.abs(Rmv - R)
    rms = (float(np.sqrt(np.mean(dA ** 2))), float(np.sqrt(np.mean(dR ** 2))))
    print(f"[mc] mean-value vs MC: max|dA| {dA.max():.3e} RMSE(A) {rms[0]:.3e} "
          f"max|dR| {dR.max():.3e} RMSE(R) {rms[1]:.3e}", flush=True)
    assert dA.max() <= hw.max() and dR.max() <= hw.max()
    # One realization of Monte Carlo noise that is correlated along the grid:
    # its RMS over the grid has the size sqrt(mean p(1-p) / M) (within a
    # factor 2), and the printed RMS values (another random stream) have the
    # same order of magnitude (within a factor 3).
    noise = (float(np.sqrt(np.mean(A * (1 - A)) / M)), float(np.sqrt(np.mean(R * (1 - R)) / M)))
    print(f"[mc] noise level sqrt(mean p(1-p)/M): A {noise[0]:.3e}, R {noise[1]:.3e}", flush=True)
    printed = dict((r[0], [float(x) for x in r[1:]]) for r in fxm["discrepancies"])["mean_value"]
    for got, lvl, pr in zip(rms, noise, (printed[1], printed[3])):
        assert 0.5 <= got / lvl <= 2.0
        assert 1 / 3 <= got / pr <= 3.0
