"""Generator checks: masses, supports, draw reproducibility."""
import math

import numpy as np
import torch

import smk_inputs as si


def test_weibull_kernel_is_a_semi_markov_kernel():
    k = si.weibull_kernel(6, 300, 1)
    q = k.q.numpy()
    assert q.shape == (300, 6, 6)
    assert np.all(q[0] == 0)
    assert q.min() >= 0
    assert np.allclose(q.sum(axis=(0, 2)), 1.0, atol=1e-13)
    assert np.all(np.diag(k.p) == 0)
    assert np.allclose(k.p.sum(1), 1.0)


def test_lognormal_kernel_mass():
    k = si.lognormal_kernel(5, 500, 3)
    q = k.q.numpy()
    assert q.min() >= 0 and np.all(q[0] == 0)
    assert np.allclose(q.sum(axis=(0, 2)), 1.0, atol=1e-12)


def test_prefix_rows_are_the_same_law():
    full = si.weibull_kernel(4, 1000, 9).q
    pre = si.weibull_kernel(4, 1000, 9, n_rows=100).q
    assert torch.equal(full[:100], pre)
    full = si.lognormal_kernel(4, 1000, 9).q
    pre = si.lognormal_kernel(4, 1000, 9, n_rows=100).q
    assert torch.equal(full[:100], pre)


def test_seed_reproducible():
    a = si.weibull_kernel(3, 50, 4).q
    b = si.weibull_kernel(3, 50, 4).q
    c = si.weibull_kernel(3, 50, 5).q
    assert torch.equal(a, b) and not torch.equal(a, c)


def test_weibull_pmf_against_survival_function():
    shape, scale, n = 1.3, 7.0, 64
    f = si.weibull_pmf(shape, scale, n).numpy()
    S = lambda t: math.exp(-((t / scale) ** shape))
    raw = np.array([0.0] + [S(k - 1) - S(k) for k in range(1, n)])
    assert np.allclose(f, raw / (1 - S(n - 1)), rtol=1e-13, atol=1e-16)


def test_geometric_not_renormalised():
    k = si.geometric_kernel(3, 20, 2)
    a = k.params["a"]
    q = k.q.numpy()
    assert np.allclose(q[1], np.diag(1 - a) @ k.p)
    assert np.allclose(q[5], np.diag((1 - a) * a ** 4) @ k.p)


def test_batch_workload_ranges():
    w = si.batch_workload()
    assert len(w) == 512
    assert all(3 <= x["d"] <= 48 for x in w)
    assert all(1024 <= x["n"] <= 32768 for x in w)
    assert {x["family"] for x in w} == {"weibull", "lognormal"}
    assert w == si.batch_workload()


def test_paper_kernels():
    k = si.paper_three_state_poisson(128)
    q = k.q.numpy()
    assert np.allclose(q.sum(axis=(0, 2)), 1.0, atol=1e-14)
    g = si.paper_three_state_gamma(2048).q.numpy()
    assert np.allclose(g.sum(axis=(0, 2)), 1.0, atol=1e-12)
    u = si.paper_uniform_poisson(4, 256).q.numpy()
    assert np.allclose(u.sum(axis=(0, 2)), 1.0, atol=1e-12)
