"""Exact rational path enumeration for tiny inputs (test infrastructure).

Independent of every recursion: by the Neumann form of Theorem 2.1 and the
renewal-sequence identity of Section 4.1, psi = sum_{m>=0} q^(m) (m-fold
convolution powers), and with q(0) = 0 the m-fold power at time k sums, over
state paths i = j_0 -> j_1 -> ... -> j_m = j and compositions
k = t_1 + ... + t_m with every t >= 1, the products q(t_1)_{j0 j1} ... q(t_m)_{j(m-1) jm}.
Terms with m > k vanish, so the sum is finite.  Everything is done with
``fractions.Fraction``; it is meant for d <= 3 and n <= 10.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product


def compositions(k: int, m: int):
    """All ordered m-tuples of integers >= 1 that sum to k."""
    if m == 0:
        if k == 0:
            yield ()
        return
    for t in range(1, k - m + 2):
        for rest in compositions(k - t, m - 1):
            yield (t,) + rest


def psi_paths(q) -> list:
    """q: nested list q[k][i][j] of Fractions with q[0] == 0. Returns psi likewise."""
    n = len(q)
    d = len(q[0])
    out = [[[Fraction(0)] * d for _ in range(d)] for _ in range(n)]
    for i in range(d):
        out[0][i][i] = Fraction(1)
    for k in range(1, n):
        for m in range(1, k + 1):
            for ts in compositions(k, m):
                for mids in product(range(d), repeat=m - 1):
                    for i in range(d):
                        for j in range(d):
                            path = (i,) + mids + (j,)
                            w = Fraction(1)
                            for s, t in enumerate(ts):
                                w *= q[t][path[s]][path[s + 1]]
                                if w == 0:
                                    break
                            if w:
                                out[k][i][j] += w
    return out


def random_rational_kernel(d: int, n: int, rng, denom: int = 7) -> list:
    """Nonnegative rational kernel with q(0) = 0 and small denominators."""
    q = [[[Fraction(0)] * d for _ in range(d)] for _ in range(n)]
    for k in range(1, n):
        for i in range(d):
            for j in range(d):
                q[k][i][j] = Fraction(int(rng.integers(0, denom)), denom * d * n)
    return q
