"""Where the FP64 bound of the long-horizon GPU tests comes from.

An independent FFT-Newton written with numpy's real FFT (a library
primitive, no code shared with the GPU path) inverts the geometric
(exact Markov) kernel of the three-pass GPU test, d = 3, n = 300000, and is
compared with the closed form psi(k) = M^(k-1)(M - diag a).  Run with the
first product A*B at the cyclic length m' (the GPU path's choice, which
halves the transform work) its error exceeds the 1e-12 target; zero-padded
to 2m' it stays well below.  The relaxed bound of tolerances.fp64_tol covers
the cyclic scheme with headroom.  The Newton iteration itself is eq. (newton)
with doubling truncation (Appendix, algorithmic details); this copy is a
test instrument only.
"""
import numpy as np
import pytest

import smk_inputs as si
from tolerances import FP64_TOL, fp64_tol


def _numpy_fft_newton(q, pad_first: bool):
    n, d, _ = q.shape
    A = -q.copy()
    A[0] += np.eye(d)
    X = np.zeros_like(A)
    X[0] = np.linalg.inv(A[0])
    m = 1
    while m < n:
        m2 = min(2 * m, n)
        L = 1
        while L < m2:
            L *= 2
        L1 = 2 * L if pad_first else L
        T = np.fft.irfft(np.matmul(np.fft.rfft(A[:m2], n=L1, axis=0), np.fft.rfft(X[:m], n=L1, axis=0)),
                         n=L1, axis=0)[:m2]
        E = np.zeros((m2, d, d))
        E[m:m2] = -T[m:m2]                    # e0 - A*X vanishes below m
        U = np.fft.irfft(np.matmul(np.fft.rfft(X[:m], n=L, axis=0), np.fft.rfft(E, n=L, axis=0)),
                         n=L, axis=0)
        X[m:m2] = U[m:m2]                     # B[m, m') = (B*E)[m, m')
        m = m2
    return X


def test_cyclic_first_product_sets_the_long_horizon_fp64_bound(orc):
    d, n = 3, 300000
    k = si.geometric_kernel(d, n, 31)
    q = k.q.numpy()
    ks = np.unique(np.concatenate([[0, 1, 2, 3, 100, 4097, 65536, 131071, 262144, n - 1],
                                   np.linspace(0, n - 1, 100).astype(int)]))
    ref = orc.geometric_psi(k.params["M"], k.params["a"], ks)
    e_cyc = float(np.max(np.abs(_numpy_fft_newton(q, False)[ks] - ref)))
    e_pad = float(np.max(np.abs(_numpy_fft_newton(q, True)[ks] - ref)))
    print(f"numpy FFT-Newton n={n}: cyclic first product {e_cyc:.2e}, padded {e_pad:.2e}, "
          f"bound {fp64_tol(n):.2e}")
    assert e_pad <= 0.5 * FP64_TOL
    assert e_cyc > FP64_TOL                 # the 1e-12 target is out of reach of this scheme
    assert e_cyc <= 0.5 * fp64_tol(n)       # the bound leaves a factor 2 over it
    # A decaying (transient) kernel has no plateau: both schemes agree to rounding.
    qt = 0.5 * q[:1 << 15]
    assert np.max(np.abs(_numpy_fft_newton(qt, False) - _numpy_fft_newton(qt, True))) <= 1e-15
