"""CPU FP64 oracle (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liborc.so`` (built from
``mrinv_oracle.c`` by :func:`build`) with numpy arrays and never touches the
GPU library.

Functions follow the paper's plain definitions (see the C source header for
the exact passages).  All arrays are float64, time-major ``[n, rows, cols]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrinv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics kept)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L = ctypes.c_long
    I = ctypes.c_int
    sig = {
        "orc_gj_inverse": (I, [dp, I, dp]),
        "orc_inverse_left_cols": (I, [dp, I, L, ip, I, dp]),
        "orc_inverse_left": (I, [dp, I, L, dp]),
        "orc_inverse_row": (I, [dp, I, L, dp, dp]),
        "orc_inverse_right": (I, [dp, I, L, dp]),
        "orc_conv": (None, [dp, dp, I, I, I, L, dp]),
        "orc_residual_at": (None, [dp, I, dp, I, ctypes.POINTER(ctypes.c_long), I, dp]),
        "orc_hbar": (None, [dp, I, L, dp]),
        "orc_transition": (None, [dp, dp, I, L, dp]),
        "orc_availability": (I, [dp, I, L, dp, ip, dp]),
        "orc_first_entrance": (I, [dp, I, L, ip, dp, dp, dp]),
        "orc_adjoint": (None, [dp, dp, I, L, dp]),
        "orc_forward_mode": (None, [dp, dp, dp, I, L, dp]),
        "orc_num_threads": (I, []),
        "orc_philox4x32_10": (None, [ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(ctypes.c_uint),
                                     ctypes.POINTER(ctypes.c_uint)]),
        "orc_semi_markov_mc": (None, [I, I, I, dp, dp, dp, ip, ctypes.c_double, L, L, ctypes.c_ulonglong,
                                      ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong), dp,
                                      ip]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class SingularError(ValueError):
    pass


def num_threads() -> int:
    return int(_load().orc_num_threads())


def gj_inverse(A0) -> np.ndarray:
    A0 = _f64(A0)
    d = A0.shape[0]
    out = np.empty_like(A0)
    if _load().orc_gj_inverse(_p(A0), d, _p(out)):
        raise SingularError("A(0) is singular")
    return out


def series_inverse_left(A, cols=None) -> np.ndarray:
    """Inverse of the sequence A on its horizon by the left recursion
    X(k) = -A(0)^-1 sum_{l>=1} A(l) X(k-l); optionally only some columns."""
    A = _f64(A)
    n, d, _ = A.shape
    if cols is None:
        out = np.empty((n, d, d))
        rc = _load().orc_inverse_left(_p(A), d, n, _p(out))
    else:
        c = np.ascontiguousarray(cols, dtype=np.int32)
        out = np.empty((n, d, len(c)))
        rc = _load().orc_inverse_left_cols(_p(A), d, n, _ip(c), len(c), _p(out))
    if rc:
        raise SingularError("A(0) is singular")
    return out


def series_inverse_right(A) -> np.ndarray:
    """Inverse by the paper's right recursion X(k) = -sum_{l<k} X(l) A(k-l) A(0)^-1."""
    A = _f64(A)
    n, d, _ = A.shape
    out = np.empty((n, d, d))
    if _load().orc_inverse_right(_p(A), d, n, _p(out)):
        raise SingularError("A(0) is singular")
    return out


def series_inverse_row(A, alpha) -> np.ndarray:
    """Row vector alpha A^-1(k), k < n, by the right recursion; returns [n, d]."""
    A = _f64(A)
    n, d, _ = A.shape
    al = _f64(alpha)
    out = np.empty((n, d))
    if _load().orc_inverse_row(_p(A), d, n, _p(al), _p(out)):
        raise SingularError("A(0) is singular")
    return out


def e0_minus(q) -> np.ndarray:
    """The sequence e0 - q."""
    q = _f64(q)
    A = -q
    A[0] += np.eye(q.shape[1])
    return A


def psi(q, cols=None) -> np.ndarray:
    """Markov renewal sequence psi = (e0 - q)^-1 (left recursion)."""
    return series_inverse_left(e0_minus(q), cols)


def psi_right(q) -> np.ndarray:
    return series_inverse_right(e0_minus(q))


def conv(A, B) -> np.ndarray:
    """Truncated convolution (A*B)(k) = sum_{l<=k} A(l) B(k-l), rectangular."""
    A = _f64(A)
    B = _f64(B)
    n, ra, m = A.shape
    assert B.shape[0] == n and B.shape[1] == m
    cb = B.shape[2]
    out = np.empty((n, ra, cb))
    _load().orc_conv(_p(A), _p(B), ra, m, cb, n, _p(out))
    return out


def hbar(q) -> np.ndarray:
    """Diagonal of the survival sequence, [n, d]."""
    q = _f64(q)
    n, d, _ = q.shape
    out = np.empty((n, d))
    _load().orc_hbar(_p(q), d, n, _p(out))
    return out


def transition(psi_seq, q) -> np.ndarray:
    """P = psi * Hbar."""
    ps = _f64(psi_seq)
    q = _f64(q)
    n, d, _ = q.shape
    out = np.empty((n, d, d))
    _load().orc_transition(_p(ps), _p(q), d, n, _p(out))
    return out


def availability(q, up, alpha=None) -> np.ndarray:
    """Occupation probability of the set ``up`` (0/1 mask): alpha P(k) 1_up."""
    q = _f64(q)
    n, d, _ = q.shape
    al = np.zeros(d) if alpha is None else _f64(alpha)
    if alpha is None:
        al[0] = 1.0
    m = np.ascontiguousarray(up, dtype=np.int32)
    out = np.empty(n)
    if _load().orc_availability(_p(q), d, n, _p(al), _ip(m), _p(out)):
        raise SingularError("singular")
    return out


def first_entrance(q, in_D, alpha=None):
    """Returns (mass ga, cdf F) of the first entrance into D from alpha on C."""
    q = _f64(q)
    n, d, _ = q.shape
    al = np.zeros(d) if alpha is None else _f64(alpha)
    m = np.ascontiguousarray(in_D, dtype=np.int32)
    if alpha is None:
        al[int(np.flatnonzero(m == 0)[0])] = 1.0
    ga = np.empty(n)
    F = np.empty(n)
    if _load().orc_first_entrance(_p(q), d, n, _ip(m), _p(al), _p(ga), _p(F)):
        raise SingularError("singular")
    return ga, F


def reliability(q, up, alpha=None) -> np.ndarray:
    """R(k) = 1 - F_D(k) with D the complement of ``up`` and alpha on ``up``."""
    up = np.asarray(up, dtype=np.int32)
    _, F = first_entrance(q, 1 - up, alpha)
    return 1.0 - F


def renewal_visits(q, inB, alpha) -> np.ndarray:
    """Expected renewal visits to B up to time k, counting the renewal at time
    zero (Section 4.1, eq. (renewal-visits)): N_B(k) = alpha sum_{l<=k} psi(l)
    I_B 1, with the row alpha psi from the right recursion.  Returns [n]."""
    q = _f64(q)
    r = series_inverse_row(e0_minus(q), _f64(alpha))
    return np.cumsum(r @ np.asarray(inB, dtype=np.float64))


def mre_mean_value(Qs, L) -> np.ndarray:
    """Mean-value (endpoint) discretisation of the continuous-time Markov
    renewal equation K = L + Q star K (Section 4.2, eqs. (mre-discrete) and
    (mre-solution)).  Qs is the kernel on the grid, Qs[m] = Q(m h) for
    m = 0..n ([n+1, d, d]); L is [n, d, r], L[m] = L(m h).  With
    Delta Q_h(0) = 0, Delta Q_h(m) = Q_h(m) - Q_h(m-1), Delta+Q_h(m) =
    Delta Q_h(m+1) and Qbar_h = (Delta Q_h + Delta+Q_h)/2:
        K_h = (e0 - Qbar_h)^(-1) * [L_h - 1/2 Delta+Q_h * (L_h(0) e0)],
    where the last product is Delta+Q_h(m) L_h(0) at every m (the sequence
    L_h(0) e0 has one coefficient).  Qbar_h(0) = Delta Q_h(1)/2, so the
    inverse has A(0) = I - Qbar_h(0) != I.  Returns K_h [n, d, r]."""
    Qs = _f64(Qs)
    L = _f64(L)
    n = L.shape[0]
    if Qs.shape[0] != n + 1:
        raise ValueError("Qs needs n + 1 grid values")
    dQ = np.zeros_like(Qs)
    dQ[1:] = Qs[1:] - Qs[:-1]
    dQp = dQ[1:n + 1]
    Qbar = 0.5 * (dQ[:n] + dQp)
    A = -Qbar
    A[0] += np.eye(Qs.shape[1])
    X = series_inverse_left(A)
    rhs = L - 0.5 * np.matmul(dQp, L[0])
    return conv(X, rhs)


def philox4x32_10(counter, key) -> np.ndarray:
    """One block of Philox4x32-10 (Salmon et al., SC 2011): four 32-bit words."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    up = ctypes.POINTER(ctypes.c_uint)
    _load().orc_philox4x32_10(c.ctypes.data_as(up), k.ctypes.data_as(up), out.ctypes.data_as(up))
    return out


FAMILIES = {"lognormal": 0, "weibull": 1, "exponential": 2}


def semi_markov_mc(P, p1, p2, up, h, n, trajectories, seed, family="lognormal", initial=0, per_path=False):
    """Pathwise Monte Carlo of a semi-Markov process on the grid m h, m < n
    (the Section 5.2 validation).  Returns (A, R) estimates, and with
    per_path also (tau_D, jumps) per trajectory; see mrinv_oracle.c for the
    stream layout and sampling."""
    P = _f64(P)
    d = P.shape[0]
    a = np.zeros(n, dtype=np.int64)
    r = np.zeros(n, dtype=np.int64)
    tau = np.empty(trajectories) if per_path else None
    jumps = np.empty(trajectories, dtype=np.int32) if per_path else None
    lp = ctypes.POINTER(ctypes.c_longlong)
    _load().orc_semi_markov_mc(d, FAMILIES[family], int(initial), _p(P), _p(_f64(p1)), _p(_f64(p2)),
                               _ip(np.ascontiguousarray(up, dtype=np.int32)), float(h), int(n), int(trajectories),
                               int(seed), a.ctypes.data_as(lp), r.ctypes.data_as(lp),
                               _p(tau) if per_path else None, _ip(jumps) if per_path else None)
    A, R = a / trajectories, r / trajectories
    return (A, R, tau, jumps) if per_path else (A, R)


def adjoint(psi_seq, psibar) -> np.ndarray:
    """qbar(b) = sum_{a+b+c<n} psi(a)^T psibar(a+b+c) psi(c)^T."""
    ps = _f64(psi_seq)
    pb = _f64(psibar)
    n, d, _ = ps.shape
    out = np.empty((n, d, d))
    _load().orc_adjoint(_p(ps), _p(pb), d, n, _p(out))
    return out


def forward_mode(q, psi_seq, dq) -> np.ndarray:
    """Directional derivative of psi along dq from psi = e0 + q*psi."""
    q = _f64(q)
    ps = _f64(psi_seq)
    dqa = _f64(dq)
    n, d, _ = q.shape
    out = np.empty((n, d, d))
    _load().orc_forward_mode(_p(q), _p(ps), _p(dqa), d, n, _p(out))
    return out


def residuals(A, X):
    """Left and right residual sequences e0 - A*X and e0 - X*A (direct)."""
    n, d, _ = A.shape
    E = np.zeros((n, d, d))
    E[0] = np.eye(d)
    return E - conv(A, X), E - conv(X, A)


def residual_at(A, X, ks, e0_minus: bool = False) -> np.ndarray:
    """Left residual e0 - A*X at the coefficients ks only, each by the direct
    sum over l = 0..k (no transform); returns [len(ks), d, d].  With e0_minus
    the first argument is q and A = e0 - q.  A and X may be longer than
    max(ks) + 1; only their first max(ks) + 1 coefficients are read."""
    A = _f64(A)
    X = _f64(X)
    n, d, _ = A.shape
    kk = np.ascontiguousarray(ks, dtype=np.int64)
    if kk.size and (kk.min() < 0 or kk.max() >= min(n, X.shape[0])):
        raise ValueError("coefficient index out of range")
    out = np.empty((kk.size, d, d))
    _load().orc_residual_at(_p(A), int(bool(e0_minus)), _p(X), d,
                            kk.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), int(kk.size), _p(out))
    return out


def norm_1N(R, spectral: bool = True) -> float:
    """||R||_{1,N} = sum_k ||R(k)||_2 (spectral; Frobenius upper bound if not)."""
    R = _f64(R)
    if spectral:
        return float(np.sum(np.linalg.norm(R, ord=2, axis=(1, 2))))
    return float(np.sum(np.linalg.norm(R, axis=(1, 2))))


def scaled_discrepancy(X, Xref, u: float = 2.0 ** -53) -> float:
    """d_N = max_k ||X(k) - Xref(k)||_F / max(||Xref(k)||_F, sqrt(u))."""
    num = np.linalg.norm(_f64(X) - _f64(Xref), axis=(1, 2))
    den = np.maximum(np.linalg.norm(_f64(Xref), axis=(1, 2)), np.sqrt(u))
    return float(np.max(num / den))


def geometric_psi(M, a, ks) -> np.ndarray:
    """Closed form for geometric sojourns (Markov chain with one-step matrix
    M = diag(a) + diag(1-a) p): psi(0) = I and psi(k) = M^(k-1) (M - diag(a))."""
    M = np.asarray(M, dtype=np.float64)
    d = M.shape[0]
    out = []
    for k in ks:
        if k == 0:
            out.append(np.eye(d))
        else:
            out.append(np.linalg.matrix_power(M, int(k) - 1) @ (M - np.diag(a)))
    return np.array(out)


def geometric_P(M, ks) -> np.ndarray:
    """Closed form P(k) = M^k of the Markov case."""
    M = np.asarray(M, dtype=np.float64)
    return np.array([np.linalg.matrix_power(M, int(k)) for k in ks])


def residuals_fft(q, X, row_block: int = 8):
    """Left/right residuals e0 - A*X and e0 - X*A (A = e0 - q) on the horizon,
    each product formed with numpy's real FFT at length >= 2n-1 (a library
    primitive independent of the GPU code), blocked over output rows.
    Returns (sum_k ||rho_L(k)||_F, sum_k ||rho_R(k)||_F, max|rho_L|, max|rho_R|)."""
    A = e0_minus(q)
    X = _f64(X)
    n, d, _ = A.shape
    Lf = 1
    while Lf < 2 * n - 1:
        Lf *= 2
    out = []
    for left, right in ((A, X), (X, A)):
        Rh = np.fft.rfft(right, n=Lf, axis=0)            # [F, d, d]
        fro2 = np.zeros(n)
        mx = 0.0
        for i0 in range(0, d, row_block):
            Lh = np.fft.rfft(left[:, i0:i0 + row_block, :], n=Lf, axis=0)
            prod = np.fft.irfft(np.matmul(Lh, Rh), n=Lf, axis=0)[:n]
            rho = -prod
            for i in range(prod.shape[1]):
                rho[0, i, i0 + i] += 1.0
            fro2 += np.sum(rho * rho, axis=(1, 2))
            mx = max(mx, float(np.max(np.abs(rho))))
        out.append((float(np.sum(np.sqrt(fro2))), mx))
    return out[0][0], out[1][0], out[0][1], out[1][1]
