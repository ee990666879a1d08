"""Seeded synthetic semi-Markov kernels.

This module only builds inputs: it draws parameters with numpy's PCG64 and
evaluates sojourn probability mass functions.  It contains none of the
inversion arithmetic, so both the GPU library and the CPU oracle may use it.

Layout of every kernel: ``q[k, i, j]`` for ``k = 0..n-1`` (time-major, one
contiguous row-major d x d matrix per time step), float64, ``q[0] = 0``.
Entry ``q[k, i, j] = p[i, j] * f_ij(k)`` is the probability of jumping from
i to j after exactly k steps (discrete semi-Markov kernel, Section 4.1).

Sojourn laws
------------
* shifted discrete Gamma ``f(k) = P(k-1 <= X < k)`` and shifted Poisson
  ``f(k) = e^-lam lam^(k-1)/(k-1)!`` (Appendix "Distributions and
  parameters"), used to replay the paper's own workloads;
* discrete Weibull and discrete lognormal with the same
  ``P(k-1 <= X < k)`` discretisation, truncated at the horizon and
  renormalised over ``k = 1..n-1``;
* geometric ``f_i(k) = (1-a_i) a_i^(k-1)`` per state (not renormalised), which
  makes the process an ordinary Markov chain.

Draw order (fixed so a seed names one kernel): rows of p (Dirichlet(1) over
the off-diagonal entries, increasing j), then the (d, d) parameter arrays
row-major, then for geometric kernels the per-state stay probabilities.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

__all__ = [
    "Kernel", "dirichlet_rows", "weibull_pmf", "lognormal_pmf", "geometric_pmf",
    "weibull_kernel", "lognormal_kernel", "geometric_kernel", "family_kernel",
    "batch_workload", "discrete_gamma_pmf", "shifted_poisson_pmf",
    "paper_three_state_gamma", "paper_three_state_poisson", "paper_uniform_poisson",
    "CONFIG_SEEDS",
]

# Seeds of the named synthetic workloads.
CONFIG_SEEDS = {"c1": 0, "c2": 1, "c2_geom": 2, "c3": 3, "c4": 4, "c5": 5}


@dataclass
class Kernel:
    q: torch.Tensor                  # [n, d, d] float64
    p: np.ndarray                    # [d, d] embedded jump matrix
    params: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return int(self.q.shape[1])

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def dirichlet_rows(rng: np.random.Generator, d: int) -> np.ndarray:
    """Row-stochastic d x d matrix, zero diagonal, Dirichlet(1) off-diagonal rows."""
    p = np.zeros((d, d))
    if d == 1:
        p[0, 0] = 1.0
        return p
    for i in range(d):
        w = rng.dirichlet(np.ones(d - 1))
        p[i, [j for j in range(d) if j != i]] = w
    return p


def _steps(n_rows: int, device) -> torch.Tensor:
    return torch.arange(n_rows, dtype=torch.float64, device=device)


def weibull_pmf(shape, scale, n: int, n_rows: int | None = None, device="cpu"):
    """Discrete Weibull mass ``S(k-1) - S(k)``, ``S(t) = exp(-(t/scale)^shape)``.

    ``shape``/``scale`` are tensors of any common shape ``B``; the result has
    shape ``[n_rows, *B]``.  ``f(0) = 0`` and the mass is renormalised over
    ``k = 1..n-1`` (division by ``1 - S(n-1)``), so rows of a kernel built from
    it sum to one over the horizon.  ``n_rows <= n`` evaluates a prefix of the
    same horizon-n law.  Differentiable in ``shape`` and ``scale``.
    """
    n_rows = n if n_rows is None else n_rows
    shape = torch.as_tensor(shape, dtype=torch.float64, device=device)
    scale = torch.as_tensor(scale, dtype=torch.float64, device=device)
    k = _steps(n_rows, device).reshape((-1,) + (1,) * shape.dim())
    km1 = torch.clamp(k - 1.0, min=0.0)

    def hazard(t):
        # (t/scale)^shape with a safe base at t = 0, so the shape derivative
        # there is 0 instead of 0 * log(0).
        pos = t > 0
        base = torch.where(pos, t, torch.ones_like(t)) / scale
        return torch.where(pos, base ** shape, torch.zeros_like(base))

    hk = hazard(k)                                  # cumulative hazard at k
    hkm1 = hazard(km1)
    f = torch.exp(-hkm1) * (-torch.expm1(-(hk - hkm1)))
    f = torch.where(k >= 1, f, torch.zeros_like(f))
    if n <= 1:
        return f
    last = torch.tensor(float(n - 1), dtype=torch.float64, device=device)
    return f / (-torch.expm1(-((last / scale) ** shape)))   # 1 - S(n-1)


def _norm_sf(z):
    return 0.5 * torch.special.erfc(z / math.sqrt(2.0))


def _norm_cdf(z):
    return 0.5 * torch.special.erfc(-z / math.sqrt(2.0))


def lognormal_pmf(mu, sigma, n: int, n_rows: int | None = None, device="cpu"):
    """Discrete lognormal mass ``Phi(z_k) - Phi(z_{k-1})``, ``z_k = (ln k - mu)/sigma``.

    ``z_0 = -inf`` so ``f(0) = 0``.  The difference is taken in the tail that
    keeps it free of cancellation (upper tail for ``z > 0``).  Renormalised
    over ``k = 1..n-1`` like :func:`weibull_pmf`.
    """
    n_rows = n if n_rows is None else n_rows
    mu = torch.as_tensor(mu, dtype=torch.float64, device=device)
    sigma = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    k = _steps(n_rows, device).reshape((-1,) + (1,) * mu.dim())
    logk = torch.log(torch.clamp(k, min=1.0))
    logkm1 = torch.log(torch.clamp(k - 1.0, min=1.0))
    zk = (logk - mu) / sigma
    zkm1 = torch.where(k >= 2, (logkm1 - mu) / sigma, torch.full_like(zk, -math.inf))
    upper = _norm_sf(zkm1) - _norm_sf(zk)
    lower = _norm_cdf(zk) - _norm_cdf(zkm1)
    f = torch.where(zk > 0, upper, lower)
    f = torch.where(k >= 1, f, torch.zeros_like(f))
    zlast = (math.log(max(n - 1, 1)) - mu) / sigma
    mass = _norm_cdf(zlast) if n > 1 else torch.ones_like(mu)
    return f / mass


def geometric_pmf(a, n_rows: int, device="cpu"):
    """``f(k) = (1-a) a^(k-1)`` for k >= 1, ``f(0) = 0``; not renormalised."""
    a = torch.as_tensor(a, dtype=torch.float64, device=device)
    k = _steps(n_rows, device).reshape((-1,) + (1,) * a.dim())
    f = (1.0 - a) * a ** torch.clamp(k - 1.0, min=0.0)
    return torch.where(k >= 1, f, torch.zeros_like(f))


def _finish(p: np.ndarray, f: torch.Tensor, device) -> torch.Tensor:
    pt = torch.as_tensor(p, dtype=torch.float64, device=device)
    q = pt.unsqueeze(0) * f
    q[0].zero_()
    return q.contiguous()


def weibull_kernel(d: int, n: int, seed: int, n_rows: int | None = None, device="cpu") -> Kernel:
    """Dirichlet(1) jump matrix; Weibull shape U[0.5, 2], scale U[2, 20] per pair."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = dirichlet_rows(rng, d)
    shape = rng.uniform(0.5, 2.0, size=(d, d))
    scale = rng.uniform(2.0, 20.0, size=(d, d))
    f = weibull_pmf(shape, scale, n, n_rows, device)
    return Kernel(_finish(p, f, device), p, {"family": "weibull", "shape": shape, "scale": scale})


def lognormal_kernel(d: int, n: int, seed: int, n_rows: int | None = None, device="cpu") -> Kernel:
    """Dirichlet(1) jump matrix; lognormal mu U[0, 3], sigma U[0.5, 2] per pair."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = dirichlet_rows(rng, d)
    mu = rng.uniform(0.0, 3.0, size=(d, d))
    sigma = rng.uniform(0.5, 2.0, size=(d, d))
    f = lognormal_pmf(mu, sigma, n, n_rows, device)
    return Kernel(_finish(p, f, device), p, {"family": "lognormal", "mu": mu, "sigma": sigma})


def geometric_kernel(d: int, n: int, seed: int, n_rows: int | None = None, device="cpu") -> Kernel:
    """Markov case: per-state stay probability a_i ~ U[0.5, 0.95].

    ``q_ij(k) = p_ij (1-a_i) a_i^(k-1)``.  The chain's one-step matrix is
    ``M = diag(a) + diag(1-a) p`` (returned in ``params['M']``).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    p = dirichlet_rows(rng, d)
    a = rng.uniform(0.5, 0.95, size=d)
    n_rows = n if n_rows is None else n_rows
    f = geometric_pmf(torch.as_tensor(a).reshape(d, 1).expand(d, d), n_rows, device)
    M = np.diag(a) + np.diag(1.0 - a) @ p
    return Kernel(_finish(p, f, device), p, {"family": "geometric", "a": a, "M": M})


def family_kernel(family: str, d: int, n: int, seed: int, **kw) -> Kernel:
    return {"weibull": weibull_kernel, "lognormal": lognormal_kernel,
            "geometric": geometric_kernel}[family](d, n, seed, **kw)


def batch_workload(seed: int = CONFIG_SEEDS["c4"], count: int = 512,
                   d_range=(3, 48), n_range=(1024, 32768)):
    """Descriptors of an uneven batch: d uniform in d_range (inclusive), n
    log-uniform in n_range, Weibull or lognormal by a fair coin, one seed each.
    Returns a list of dicts ``{d, n, family, seed}``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    for _ in range(count):
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        n = int(round(math.exp(rng.uniform(lo, hi))))
        fam = "weibull" if rng.random() < 0.5 else "lognormal"
        s = int(rng.integers(0, 2**62))
        out.append({"d": d, "n": n, "family": fam, "seed": s})
    return out


# ---------------------------------------------------------------------------
# The paper's own small workloads (Section 5.1 and the parameter appendix).
# ---------------------------------------------------------------------------

def discrete_gamma_pmf(alpha: float, theta: float, n: int) -> np.ndarray:
    """Shifted discrete Gamma ``f(k) = P(k-1 <= X < k)``, k >= 1, f(0) = 0 (not renormalised)."""
    from scipy.special import gammainc
    k = np.arange(n, dtype=np.float64)
    cdf_k = gammainc(alpha, k / theta)
    cdf_km1 = gammainc(alpha, np.maximum(k - 1, 0) / theta)
    f = cdf_k - cdf_km1
    f[0] = 0.0
    return f


def shifted_poisson_pmf(lam: float, n: int) -> np.ndarray:
    """``f(k) = e^-lam lam^(k-1)/(k-1)!`` for k >= 1, f(0) = 0."""
    from scipy.special import gammaln
    k = np.arange(n, dtype=np.float64)
    f = np.zeros(n)
    km1 = k[1:] - 1
    f[1:] = np.exp(-lam + km1 * math.log(lam) - gammaln(km1 + 1))
    return f


# Embedded chain of the three-state model (normal, degraded, shutdown).
PAPER_PEMB3 = np.array([[0.0, 1.0, 0.0], [0.2, 0.0, 0.8], [1.0, 0.0, 0.0]])


def paper_three_state_gamma(n: int) -> Kernel:
    """Horizon-scaling model: Gamma (shape, scale) = (1.8,4), (1.6,5), (2.2,4),
    (1.9,3) for 1->2, 2->1, 2->3, 3->1 (zero-based pairs below)."""
    pars = {(0, 1): (1.8, 4.0), (1, 0): (1.6, 5.0), (1, 2): (2.2, 4.0), (2, 0): (1.9, 3.0)}
    q = np.zeros((n, 3, 3))
    for (i, j), (a, t) in pars.items():
        q[:, i, j] = PAPER_PEMB3[i, j] * discrete_gamma_pmf(a, t, n)
    return Kernel(torch.from_numpy(q), PAPER_PEMB3.copy(), {"family": "gamma", "pars": pars})


def paper_three_state_poisson(n: int) -> Kernel:
    """First-entrance model: shifted Poisson lambda = 8, 5, 10, 7 for
    1->2, 2->1, 2->3, 3->1."""
    pars = {(0, 1): 8.0, (1, 0): 5.0, (1, 2): 10.0, (2, 0): 7.0}
    q = np.zeros((n, 3, 3))
    for (i, j), lam in pars.items():
        q[:, i, j] = PAPER_PEMB3[i, j] * shifted_poisson_pmf(lam, n)
    return Kernel(torch.from_numpy(q), PAPER_PEMB3.copy(), {"family": "poisson", "pars": pars})


def paper_uniform_poisson(s: int, n: int) -> Kernel:
    """State-dimension model: uniform jumps to the other states, shifted
    Poisson with lambda_ij = 3 + ((i + j) mod 4), states numbered from one."""
    p = np.full((s, s), 1.0 / (s - 1))
    np.fill_diagonal(p, 0.0)
    q = np.zeros((n, s, s))
    for i in range(s):
        for j in range(s):
            if i != j:
                q[:, i, j] = p[i, j] * shifted_poisson_pmf(3.0 + ((i + 1 + j + 1) % 4), n)
    return Kernel(torch.from_numpy(q), p, {"family": "poisson_uniform"})



def exponential_semi_markov(G: np.ndarray, h: float, count: int):
    """Exponential semi-Markov model of a generator G (Section 5.2) sampled on
    the grid t_m = m h, m = 0 .. count - 1.

    The embedded matrix is P_ij = G_ij / lambda_i (i != j) with lambda_i = -G_ii;
    the kernel is Q_ij(t) = P_ij (1 - exp(-lambda_i t)) and the survival is
    Hbar(t) = diag(exp(-lambda_i t)).  Returns (Q [count, s, s],
    Hbar [count, s, s]), both float64 numpy arrays."""
    G = np.asarray(G, dtype=np.float64)
    s = G.shape[0]
    lam = -np.diag(G)
    pemb = G / lam[:, None]
    np.fill_diagonal(pemb, 0.0)
    t = h * np.arange(count)
    Q = pemb[None] * -np.expm1(-lam[None, :, None] * t[:, None, None])
    Hbar = np.exp(-lam[None, :] * t[:, None])[:, :, None] * np.eye(s)
    return Q, Hbar


def lognormal_semi_markov(pemb, mu, sigma, h: float, count: int):
    """Lognormal semi-Markov model (Section 5.2 and the parameter appendix)
    sampled on the grid t_m = m h, m = 0 .. count - 1: the kernel
    Q_ij(t) = P_ij Phi((ln t - mu_ij) / sigma_ij) for t > 0, Q(0) = 0, and the
    survival Hbar(t) = diag(1 - sum_j Q_ij(t)).  Entries with P_ij = 0 may
    carry any mu, sigma > 0.  Returns (Q [count, s, s], Hbar [count, s, s])."""
    pemb = np.asarray(pemb, dtype=np.float64)
    s = pemb.shape[0]
    t = torch.as_tensor(h * np.arange(1, count), dtype=torch.float64)
    z = (torch.log(t)[:, None, None] - torch.as_tensor(mu, dtype=torch.float64)) / torch.as_tensor(
        sigma, dtype=torch.float64)
    Q = np.zeros((count, s, s))
    Q[1:] = pemb[None] * _norm_cdf(z).numpy()
    Hbar = (1.0 - Q.sum(axis=2))[:, :, None] * np.eye(s)
    return Q, Hbar

# ---------------------------------------------------------------------------
# Differentiable parameterisation (input construction for gradient studies).
# ---------------------------------------------------------------------------

def weibull_params(d: int, seed: int, device="cpu"):
    """Draws of :func:`weibull_kernel` as tensors (shape, scale, logits), with
    logits = log p off the diagonal (so the masked softmax reproduces p)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = dirichlet_rows(rng, d)
    shape = rng.uniform(0.5, 2.0, size=(d, d))
    scale = rng.uniform(2.0, 20.0, size=(d, d))
    logits = np.where(np.eye(d) > 0, 0.0, np.log(np.where(p > 0, p, 1.0)))
    f64 = dict(dtype=torch.float64, device=device)
    return torch.tensor(shape, **f64), torch.tensor(scale, **f64), torch.tensor(logits, **f64)


def masked_softmax_rows(logits: torch.Tensor) -> torch.Tensor:
    """Row-wise softmax over the off-diagonal entries; zero diagonal."""
    d = logits.shape[0]
    mask = torch.eye(d, dtype=torch.bool, device=logits.device)
    z = logits.masked_fill(mask, float("-inf"))
    return torch.softmax(z, dim=1)


def weibull_kernel_from_params(shape: torch.Tensor, scale: torch.Tensor, logits: torch.Tensor, n: int):
    """q(k) = softmax_offdiag(logits) * Weibull pmf(k; shape, scale); differentiable."""
    p = masked_softmax_rows(logits)
    f = weibull_pmf(shape, scale, n, device=shape.device)
    return p.unsqueeze(0) * f
