"""Parity bounds shared by the GPU tests, and the reason for each.

FP64: max-abs error <= 1e-12 against the oracle up to horizon 2^16.  The
Newton steps form their first product A*B at the cyclic length m' (the
wrap-around lands only on the discarded coefficients below m), which halves
the transform work of the padded length 2m'.  On recurrent kernels (renewal
sequences with a non-decaying plateau) that product's rounding error grows
about linearly with the coefficient index: an independent numpy FFT-Newton
with the same cyclic first product reaches 2.6e-12 at n = 300000, the padded
one 2.3e-13 (tests/test_tolerance.py runs both).  Beyond 2^16 the bound is
therefore scaled by sqrt(L / 2^16) * log2(L) / 16 with a factor 2 of headroom.

Mixed: max-abs error <= 1e-10 (the float32 Newton followed by float64
residual sweeps).
"""
import math

FP64_TOL = 1e-12
MIXED_TOL = 1e-10


def fp64_tol(n: int) -> float:
    lg = max(1, math.ceil(math.log2(n)))
    if lg <= 16:
        return FP64_TOL
    return 2 * FP64_TOL * math.sqrt(2.0 ** (lg - 16)) * lg / 16
