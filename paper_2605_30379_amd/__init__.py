"""mrinv — finite-horizon psi inversion and Markov renewal functionals on MI355X.

Thin binding over the C-ABI library ``libmrinv.so`` (declared in
``include/mrinv.h``): every function here only checks arguments, allocates
outputs and workspace with torch on the tensor's device, and passes raw
device pointers and the current HIP stream to the library.  All arithmetic
runs in the library's HIP kernels.  There is no CPU fallback: without the
built library or a GPU every call raises.

Main entry points (Kordalis & Trevezas, Sections 2 and 4):

* :func:`psi_inverse` — psi = (e0 - q)^-1 on the horizon (FP64 or mixed).
* :func:`transition` — P = psi * Hbar.
* :func:`markov_renewal_apply` — M = psi * L (reward / first-entrance kernels).
* :func:`first_entrance`, :func:`reliability`, :func:`availability`.
* :class:`PsiInverse`, :class:`RenewalApply`, :class:`Transition`,
  :class:`Contract`, :class:`GatherBlock` — autograd Functions backed by the
  library's adjoint kernels.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

__all__ = [
    "MrinvError", "lib", "library_path", "psi_inverse", "series_inverse", "markov_renewal_apply",
    "transition", "survival", "first_entrance", "reliability", "availability", "contract",
    "gather_block", "psi_inverse_backward", "markov_renewal_apply_backward", "transition_backward",
    "contract_backward", "scatter_block_add", "psi_inverse_batched", "residual_norms", "sync_status",
    "PsiInverse", "RenewalApply", "Transition", "Contract", "GatherBlock", "workspace_size",
    "FP64", "MIXED_FP32", "MIXED_BF16X3", "FP64_PADDED", "OPS", "Tuning", "get_tuning", "set_tuning", "autotune", "BatchedPlan",
    "psi_inverse_noalloc", "NOALLOC_SCRATCH_BYTES", "renewal_visits", "mre_solve",
    "series_inverse_gj", "semi_markov_mc", "McModel", "SOJOURN", "TuningEntry", "set_tuning_table",
    "load_tuning_table", "TUNING_TABLE",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmrinv.so")

FP64 = 0
MIXED_FP32 = 1
MIXED_BF16X3 = 2
FP64_PADDED = 3
_PREC = {"fp64": FP64, "mixed": MIXED_FP32, "mixed_fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3,
         "mixed_bf16x3": MIXED_BF16X3, "fp64_padded": FP64_PADDED,
         FP64: FP64, MIXED_FP32: MIXED_FP32, MIXED_BF16X3: MIXED_BF16X3, FP64_PADDED: FP64_PADDED}
OPS = {"psi_inverse": 0, "apply": 1, "transition": 2, "psi_backward": 3, "apply_backward": 4,
       "transition_backward": 5, "first_entrance": 6, "availability": 7, "residual": 8, "mre": 9, "gj": 10}

_STATUS = {0: "ok", 1: "invalid argument", 2: "A(0) singular", 3: "non-finite value",
           4: "workspace too small", 5: "unsupported size", 6: "HIP runtime error"}


class Tuning(ctypes.Structure):
    """Launch-shape and schedule choices of a handle (mrinv_tuning_t)."""
    _fields_ = [("lgp_max", ctypes.c_int), ("lanes_fp64", ctypes.c_int), ("lanes_fp32", ctypes.c_int),
                ("seed_m0", ctypes.c_int), ("pair_forward", ctypes.c_int), ("twiddle_tables", ctypes.c_int),
                ("block_order", ctypes.c_int), ("use_graph", ctypes.c_int), ("mfma", ctypes.c_int),
                ("direct_m", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class McModel(ctypes.Structure):
    """mrinv_mc_model_t."""
    _fields_ = [("d", ctypes.c_int), ("family", ctypes.c_int), ("initial", ctypes.c_int),
                ("P", ctypes.POINTER(ctypes.c_double)), ("p1", ctypes.POINTER(ctypes.c_double)),
                ("p2", ctypes.POINTER(ctypes.c_double)), ("up", ctypes.POINTER(ctypes.c_int))]


class TuningEntry(ctypes.Structure):
    """mrinv_tuning_entry_t: a tuning for problems with d in [d_lo, d_hi],
    n in [n_lo, n_hi] and the given precision (-1: any)."""
    _fields_ = [("d_lo", ctypes.c_int), ("d_hi", ctypes.c_int), ("n_lo", ctypes.c_int64), ("n_hi", ctypes.c_int64),
                ("precision", ctypes.c_int), ("tune", Tuning)]


class MrinvError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"mrinv: {_STATUS.get(status, status)} ({detail})")
        self.status = status


_lib = None
_lock = threading.Lock()
_handles: dict = {}


def lib():
    """Load libmrinv.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(library_path):
            raise MrinvError(6, f"{library_path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(library_path)
        vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        sigs = {
            "mrinv_create": (i32, [ctypes.POINTER(vp), vp]),
            "mrinv_destroy": (i32, [vp]),
            "mrinv_set_stream": (i32, [vp, vp]),
            "mrinv_sync_status": (i32, [vp]),
            "mrinv_status_string": (ctypes.c_char_p, [i32]),
            "mrinv_last_error": (ctypes.c_char_p, []),
            "mrinv_workspace_size": (sz, [i32, i32, i64, i32, i32]),
            "mrinv_psi_inverse": (i32, [vp, vp, i32, i64, i32, vp, vp, sz]),
            "mrinv_series_inverse": (i32, [vp, vp, i32, i64, i32, vp, vp, sz]),
            "mrinv_psi_inverse_noalloc": (i32, [vp, vp, i32, i64, i32, vp]),
            "mrinv_markov_renewal_apply": (i32, [vp, vp, i32, i64, vp, i32, vp, vp, sz]),
            "mrinv_transition": (i32, [vp, vp, vp, i32, i64, vp, vp, sz]),
            "mrinv_survival": (i32, [vp, vp, i32, i64, vp]),
            "mrinv_contract": (i32, [vp, vp, i64, i32, i32, vp, vp, i32, f64, f64, vp]),
            "mrinv_gather_block": (i32, [vp, vp, i64, i32, i32, vp, i32, vp, i32, vp]),
            "mrinv_first_entrance": (i32, [vp, vp, i32, i64, ip, dp, i32, vp, vp, vp, sz]),
            "mrinv_reliability": (i32, [vp, vp, i32, i64, ip, dp, i32, vp, vp, sz]),
            "mrinv_availability": (i32, [vp, vp, i32, i64, ip, dp, vp]),
            "mrinv_renewal_visits": (i32, [vp, vp, i32, i64, ip, dp, vp]),
            "mrinv_series_inverse_gj": (i32, [vp, vp, i32, i64, vp, vp, sz]),
            "mrinv_mc_workspace_size": (sz, [i64]),
            "mrinv_semi_markov_mc": (i32, [vp, ctypes.POINTER(McModel), f64, i64, i64, ctypes.c_uint64, vp, vp, vp,
                                           vp, vp, sz]),
            "mrinv_psi_inverse_gj": (i32, [vp, vp, i32, i64, vp, vp, sz]),
            "mrinv_mre_solve": (i32, [vp, vp, i32, i64, vp, i32, i32, vp, vp, sz]),
            "mrinv_psi_inverse_backward": (i32, [vp, vp, vp, i32, i64, vp, vp, sz]),
            "mrinv_markov_renewal_apply_backward": (i32, [vp, vp, vp, vp, i32, i64, i32, vp, vp, vp, sz]),
            "mrinv_transition_backward": (i32, [vp, vp, vp, vp, i32, i64, vp, vp, vp, sz]),
            "mrinv_contract_backward": (i32, [vp, vp, i64, i32, i32, vp, vp, i32, f64, vp]),
            "mrinv_scatter_block_add": (i32, [vp, vp, i64, i32, i32, vp, i32, vp, i32, vp]),
            "mrinv_psi_inverse_batched": (i32, [vp, i32, ctypes.POINTER(vp), ip, ctypes.POINTER(i64), i32,
                                                ctypes.POINTER(vp), vp, sz]),
            "mrinv_psi_inverse_batched_prepare": (i32, [vp, i32, ctypes.POINTER(vp), ip, ctypes.POINTER(i64), i32,
                                                        ctypes.POINTER(vp), vp, sz]),
            "mrinv_psi_inverse_batched_launch": (i32, [vp]),
            "mrinv_batched_workspace_size": (sz, [vp, i32, ip, ctypes.POINTER(i64), i32]),
            "mrinv_residual_norms": (i32, [vp, vp, vp, i32, i64, dp, vp, sz]),
            "mrinv_get_tuning": (i32, [vp, ctypes.POINTER(Tuning)]),
            "mrinv_set_tuning_table": (i32, [vp, ctypes.POINTER(TuningEntry), i32]),
            "mrinv_set_tuning": (i32, [vp, ctypes.POINTER(Tuning)]),
            "mrinv_autotune": (i32, [vp, vp, i32, i64, i32, vp, vp, sz, ctypes.POINTER(Tuning)]),
            "mrinv_hbm_probe": (i32, [vp, vp, sz, i32, i32, i32, dp]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def _check(status: int):
    if status != 0:
        detail = lib().mrinv_last_error().decode(errors="replace")
        raise MrinvError(status, detail)


def _handle(device: torch.device):
    """The library handle of (device, torch's current stream on it).

    A handle's scratch area is used in stream order, so each stream gets its
    own handle (the library's contract: one handle per stream).  Handles live
    until the process ends.  mrinv_create allocates and waits for the device:
    a stream that is being captured into a graph must have made one call
    before the capture."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    L = lib()
    key = (idx, stream)
    h = _handles.get(key)
    if h is None:
        with _lock:
            h = _handles.get(key)
            if h is None:
                with torch.cuda.device(idx):
                    hv = ctypes.c_void_p()
                    _check(L.mrinv_create(ctypes.byref(hv), ctypes.c_void_p(stream)))
                h = hv
                _handles[key] = h
    return h


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _seq(x: torch.Tensor, name: str, rows=None, cols=None, n=None) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.device.type != "cuda":
        raise MrinvError(1, f"{name} must be a GPU tensor (no CPU path)")
    if x.dtype != torch.float64:
        raise MrinvError(1, f"{name} must be float64")
    if x.dim() != 3:
        raise MrinvError(1, f"{name} must have shape [n, rows, cols]")
    if rows is not None and x.shape[1] != rows or cols is not None and x.shape[2] != cols:
        raise MrinvError(1, f"{name} has shape {tuple(x.shape)}")
    if n is not None and x.shape[0] != n:
        raise MrinvError(1, f"{name} has horizon {x.shape[0]}, expected {n}")
    return x.contiguous()


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def workspace_size(op: str, d: int, n: int, r: int = 0, precision="fp64") -> int:
    return int(lib().mrinv_workspace_size(OPS[op], d, n, r, _PREC[precision]))


def get_tuning(device=None) -> dict:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    t = Tuning()
    _check(lib().mrinv_get_tuning(_handle(dev), ctypes.byref(t)))
    return t.as_dict()


def set_tuning(device=None, **kw):
    """Change tuning fields of the device's handle (the fields of mrinv_tuning_t:
    lgp_max, lanes_fp64, lanes_fp32, seed_m0, pair_forward, twiddle_tables,
    block_order, use_graph, mfma, direct_m); unknown names raise."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    t = Tuning()
    h = _handle(dev)
    _check(lib().mrinv_get_tuning(h, ctypes.byref(t)))
    names = {f for f, _ in Tuning._fields_}
    for k, v in kw.items():
        if k not in names:
            raise MrinvError(1, f"unknown tuning field {k!r}")
        setattr(t, k, int(v))
    _check(lib().mrinv_set_tuning(h, ctypes.byref(t)))


TUNING_TABLE = os.path.join(_HERE, "tuning_table.json")


def set_tuning_table(entries, device=None) -> int:
    """Install a per-class tuning table in the handle of (device, current
    stream): a list of dicts with d_lo, d_hi, n_lo, n_hi, precision (a name
    such as "fp64", or -1 for any) and tune (a dict of mrinv_tuning_t fields;
    missing fields keep the handle's value).  An empty list clears it."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _handle(dev)
    base = Tuning()
    _check(lib().mrinv_get_tuning(h, ctypes.byref(base)))
    arr = (TuningEntry * max(1, len(entries)))()
    names = {f for f, _ in Tuning._fields_}
    for i, e in enumerate(entries):
        t = Tuning(*[getattr(base, f) for f, _ in Tuning._fields_])
        for k, v in e.get("tune", {}).items():
            if k not in names:
                raise MrinvError(1, f"unknown tuning field {k!r}")
            setattr(t, k, int(v))
        prec = e.get("precision", -1)
        arr[i] = TuningEntry(int(e["d_lo"]), int(e["d_hi"]), int(e["n_lo"]), int(e["n_hi"]),
                             -1 if prec in (-1, None, "any") else _PREC[prec], t)
    _check(lib().mrinv_set_tuning_table(h, arr, len(entries)))
    return len(entries)


def load_tuning_table(path: str | None = None, device=None) -> int:
    """Install the table written by paper_2605_30379_amd/tune_table.py (by
    default the one next to this file); returns the number of entries, 0 if
    there is no table."""
    import json
    path = TUNING_TABLE if path is None else path
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    return set_tuning_table(data["entries"], device)


def autotune(q: torch.Tensor, precision="fp64") -> dict:
    """Measure candidate tunings on q, keep the fastest in the device's handle."""
    q = _seq(q, "q")
    n, d, _ = q.shape
    prec = _PREC[precision]
    out = torch.empty_like(q)
    ws = _ws(lib().mrinv_workspace_size(0, d, n, 0, prec), q.device)
    t = Tuning()
    _check(lib().mrinv_autotune(_handle(q.device), _ptr(q), d, n, prec, _ptr(out), _ptr(ws), ws.numel(),
                                ctypes.byref(t)))
    return t.as_dict()


HBM_PATTERNS = {"copy": 0, "pass_first": 1, "pass_last": 2}


def hbm_probe(buf: torch.Tensor, pattern="copy", lanes: int = 16, reps: int = 5) -> float:
    """Best read + write rate (GB/s) of one access pattern over the device
    buffer `buf` (contents overwritten; mrinv_hbm_probe)."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise MrinvError(1, "buf must be a contiguous device tensor")
    out = ctypes.c_double(0.0)
    _check(lib().mrinv_hbm_probe(_handle(buf.device), _ptr(buf), buf.numel() * buf.element_size(),
                                 HBM_PATTERNS[pattern], int(lanes), int(reps), ctypes.byref(out)))
    return out.value


def sync_status(device=None):
    """Synchronise and raise if a device-side condition was flagged."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    _check(lib().mrinv_sync_status(_handle(dev)))


# ---------------------------------------------------------------------------
# Forward entry points
# ---------------------------------------------------------------------------

def psi_inverse(q: torch.Tensor, precision="fp64", check: bool = False) -> torch.Tensor:
    """psi = (e0 - q)^-1 on the horizon n = q.shape[0] (eq. (renewal-sequence))."""
    q = _seq(q, "q")
    n, d, d2 = q.shape
    if d != d2:
        raise MrinvError(1, "q must be square")
    prec = _PREC[precision]
    out = torch.empty_like(q)
    ws = _ws(lib().mrinv_workspace_size(0, d, n, 0, prec), q.device)
    _check(lib().mrinv_psi_inverse(_handle(q.device), _ptr(q), d, n, prec, _ptr(out), _ptr(ws), ws.numel()))
    if check:
        sync_status(q.device)
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def psi_inverse_noalloc(q: torch.Tensor, psi: torch.Tensor, precision="fp64") -> torch.Tensor:
    """psi_inverse into a caller-given output with the library-owned workspace
    (mrinv_psi_inverse_noalloc): nothing is allocated, by this function or the
    library.  The handle of the stream must exist (make one call on the
    stream first).  Calls overlapping on one GPU race; see include/mrinv.h."""
    q = _square(q, "q")
    n, d, _ = q.shape
    if not isinstance(psi, torch.Tensor) or psi.shape != q.shape or psi.dtype != torch.float64 \
            or not psi.is_contiguous() or psi.device != q.device:
        raise MrinvError(1, "psi must be a contiguous float64 tensor shaped like q on its device")
    _check(lib().mrinv_psi_inverse_noalloc(_handle(q.device), _ptr(q), d, n, _PREC[precision], _ptr(psi)))
    return psi


def series_inverse(A: torch.Tensor, precision="fp64", check: bool = False) -> torch.Tensor:
    """A^(-1) on the horizon for a general sequence with A(0) nonsingular (Theorem 2.1)."""
    A = _seq(A, "A")
    n, d, d2 = A.shape
    if d != d2:
        raise MrinvError(1, "A must be square")
    prec = _PREC[precision]
    out = torch.empty_like(A)
    ws = _ws(lib().mrinv_workspace_size(0, d, n, 0, prec), A.device)
    _check(lib().mrinv_series_inverse(_handle(A.device), _ptr(A), d, n, prec, _ptr(out), _ptr(ws), ws.numel()))
    if check:
        sync_status(A.device)
    return out


def series_inverse_gj(A: torch.Tensor, check: bool = False, e0_minus: bool = False) -> torch.Tensor:
    """A^(-1) on the horizon by Gauss-Jordan elimination over the truncated
    series ring (Appendix); with e0_minus the argument is q and the result is
    psi = (e0 - q)^(-1).  FP64."""
    A = _square(A, "A")
    n, d, _ = A.shape
    out = torch.empty_like(A)
    ws = _ws(lib().mrinv_workspace_size(10, d, n, 0, 0), A.device)
    fn = lib().mrinv_psi_inverse_gj if e0_minus else lib().mrinv_series_inverse_gj
    _check(fn(_handle(A.device), _ptr(A), d, n, _ptr(out), _ptr(ws), ws.numel()))
    if check:
        sync_status(A.device)
    return out


def markov_renewal_apply(psi: torch.Tensor, L: torch.Tensor) -> torch.Tensor:
    """M = psi * L truncated at n (L: [n, d, r])."""
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    L = _seq(L, "L", rows=d, n=n)
    r = L.shape[2]
    M = torch.empty_like(L)
    ws = _ws(lib().mrinv_workspace_size(1, d, n, r, 0), psi.device)
    _check(lib().mrinv_markov_renewal_apply(_handle(psi.device), _ptr(psi), d, n, _ptr(L), r, _ptr(M), _ptr(ws),
                                            ws.numel()))
    return M


def transition(psi: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """P = psi * Hbar(q) (eq. (transition-discrete))."""
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    q = _seq(q, "q", d, d, n=n)
    P = torch.empty_like(psi)
    ws = _ws(lib().mrinv_workspace_size(2, d, n, 0, 0), psi.device)
    _check(lib().mrinv_transition(_handle(psi.device), _ptr(psi), _ptr(q), d, n, _ptr(P), _ptr(ws), ws.numel()))
    return P


def survival(q: torch.Tensor) -> torch.Tensor:
    """Diagonal of Hbar: [n, d]."""
    q = _square(q, "q")
    n, d, _ = q.shape
    hb = torch.empty((n, d), dtype=torch.float64, device=q.device)
    _check(lib().mrinv_survival(_handle(q.device), _ptr(q), d, n, _ptr(hb)))
    return hb


def _dvec(v, n, device, dtype=torch.float64):
    t = torch.as_tensor(v, dtype=dtype).reshape(-1)
    if t.numel() != n:
        raise MrinvError(1, f"vector of length {t.numel()} != {n}")
    return t.to(device).contiguous()


def contract(X: torch.Tensor, u, v, cumulative: bool = False, offset: float = 0.0, scale: float = 1.0):
    """out(k) = offset + scale * u^T X(k) v (cumulative: summed over l <= k)."""
    X = _seq(X, "X")
    n, r, c = X.shape
    u = _dvec(u, r, X.device)
    v = _dvec(v, c, X.device)
    out = torch.empty(n, dtype=torch.float64, device=X.device)
    _check(lib().mrinv_contract(_handle(X.device), _ptr(X), n, r, c, _ptr(u), _ptr(v), int(cumulative),
                                float(offset), float(scale), _ptr(out)))
    return out


def _indices(idx, bound: int, name: str, distinct: bool = False) -> torch.Tensor:
    t = torch.as_tensor(idx, dtype=torch.int64).reshape(-1)
    if t.numel() < 1:
        raise MrinvError(1, f"{name} is empty")
    if int(t.min()) < 0 or int(t.max()) >= bound:
        raise MrinvError(1, f"{name} has an index outside [0, {bound})")
    if distinct and torch.unique(t).numel() != t.numel():
        raise MrinvError(1, f"{name} has repeated indices")
    return t.to(torch.int32)


def gather_block(X: torch.Tensor, rows_idx, cols_idx) -> torch.Tensor:
    X = _seq(X, "X")
    n, r, c = X.shape
    rows_idx = _indices(rows_idx, r, "rows_idx")
    cols_idx = _indices(cols_idx, c, "cols_idx")
    ri = torch.as_tensor(rows_idx, dtype=torch.int32).to(X.device).contiguous()
    ci = torch.as_tensor(cols_idx, dtype=torch.int32).to(X.device).contiguous()
    Y = torch.empty((n, ri.numel(), ci.numel()), dtype=torch.float64, device=X.device)
    _check(lib().mrinv_gather_block(_handle(X.device), _ptr(X), n, r, c, _ptr(ri), ri.numel(), _ptr(ci),
                                    ci.numel(), _ptr(Y)))
    return Y


def _imask(m, d):
    arr = (ctypes.c_int * d)(*[int(bool(x)) for x in list(m)])
    return arr


def _dalpha(alpha, d):
    if alpha is None:
        raise MrinvError(1, "alpha is required")
    vals = [float(x) for x in torch.as_tensor(alpha, dtype=torch.float64).reshape(-1).tolist()]
    if len(vals) != d:
        raise MrinvError(1, "alpha must have length d")
    return (ctypes.c_double * d)(*vals)


def first_entrance(q: torch.Tensor, in_D, alpha, precision="fp64"):
    """(g, F): first-entrance mass alpha_C g_D(k) 1_D and cdf F_D(k) (eqs. (first-entrance-mass, -cdf))."""
    q = _square(q, "q")
    n, d, _ = q.shape
    mask = [int(bool(x)) for x in list(in_D)]
    prec = _PREC[precision]
    g = torch.empty(n, dtype=torch.float64, device=q.device)
    F = torch.empty(n, dtype=torch.float64, device=q.device)
    ws = _ws(lib().mrinv_workspace_size(6, d, n, max(1, sum(mask)), prec), q.device)
    _check(lib().mrinv_first_entrance(_handle(q.device), _ptr(q), d, n, _imask(mask, d), _dalpha(alpha, d), prec,
                                      _ptr(g), _ptr(F), _ptr(ws), ws.numel()))
    return g, F


def reliability(q: torch.Tensor, up, alpha, precision="fp64") -> torch.Tensor:
    """R(k) = 1 - F_D(k) with D the complement of the up set."""
    q = _square(q, "q")
    n, d, _ = q.shape
    mask = [int(bool(x)) for x in list(up)]
    prec = _PREC[precision]
    R = torch.empty(n, dtype=torch.float64, device=q.device)
    ws = _ws(lib().mrinv_workspace_size(6, d, n, max(1, d - sum(mask)), prec), q.device)
    _check(lib().mrinv_reliability(_handle(q.device), _ptr(q), d, n, _imask(mask, d), _dalpha(alpha, d), prec,
                                   _ptr(R), _ptr(ws), ws.numel()))
    return R


def availability(P: torch.Tensor, up, alpha) -> torch.Tensor:
    """A(k) = alpha P(k) 1_U."""
    P = _square(P, "P")
    n, d, _ = P.shape
    A = torch.empty(n, dtype=torch.float64, device=P.device)
    _check(lib().mrinv_availability(_handle(P.device), _ptr(P), d, n, _imask(up, d), _dalpha(alpha, d), _ptr(A)))
    return A


def renewal_visits(psi: torch.Tensor, in_B, alpha) -> torch.Tensor:
    """N_B(k) = alpha sum_{l<=k} psi(l) I_B 1 (eq. (renewal-visits))."""
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    N = torch.empty(n, dtype=torch.float64, device=psi.device)
    _check(lib().mrinv_renewal_visits(_handle(psi.device), _ptr(psi), d, n, _imask(in_B, d), _dalpha(alpha, d),
                                      _ptr(N)))
    return N


def mre_solve(Qs: torch.Tensor, L: torch.Tensor, precision="fp64") -> torch.Tensor:
    """Mean-value discretisation of K = L + Q (Stieltjes) K (Section 4.2,
    eq. (mre-solution)): Qs [n+1, d, d] is Q on the grid t_m = m h, L [n, d, r]
    is L(t_m); returns K_h [n, d, r]."""
    Qs = _square(Qs, "Qs")
    n1, d, _ = Qs.shape
    n = n1 - 1
    if n < 1:
        raise MrinvError(1, "Qs needs at least two grid values")
    L = _seq(L, "L", rows=d, n=n)
    r = L.shape[2]
    prec = _PREC[precision]
    K = torch.empty_like(L)
    ws = _ws(lib().mrinv_workspace_size(9, d, n, r, prec), Qs.device)
    _check(lib().mrinv_mre_solve(_handle(Qs.device), _ptr(Qs), d, n, _ptr(L), r, prec, _ptr(K), _ptr(ws),
                                 ws.numel()))
    return K


SOJOURN = {"lognormal": 0, "weibull": 1, "exponential": 2}


def semi_markov_mc(P, p1, p2, up, step: float, n: int, trajectories: int, seed: int, family="lognormal",
                   initial: int = 0, per_path: bool = False, device=None):
    """Pathwise Monte Carlo of a semi-Markov process (mrinv_semi_markov_mc):
    availability and reliability estimates on the grid m*step, m < n, as
    float64 tensors on the GPU; with per_path also the first entrance time
    into the down set and the number of jumps of every trajectory."""
    import numpy as np
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    P_ = np.ascontiguousarray(P, dtype=np.float64)
    d = P_.shape[0]
    a1 = np.ascontiguousarray(p1, dtype=np.float64)
    a2 = np.ascontiguousarray(p2, dtype=np.float64)
    um = np.ascontiguousarray(up, dtype=np.int32)
    if P_.shape != (d, d) or a1.shape != (d, d) or a2.shape != (d, d) or um.shape != (d,):
        raise MrinvError(1, "P, p1, p2 must be d x d and up of length d")
    dp = ctypes.POINTER(ctypes.c_double)
    m = McModel(d, SOJOURN[family], int(initial), P_.ctypes.data_as(dp), a1.ctypes.data_as(dp),
                a2.ctypes.data_as(dp), um.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    A = torch.empty(n, dtype=torch.float64, device=dev)
    R = torch.empty(n, dtype=torch.float64, device=dev)
    tau = torch.empty(trajectories, dtype=torch.float64, device=dev) if per_path else None
    jumps = torch.empty(trajectories, dtype=torch.int32, device=dev) if per_path else None
    L = lib()
    ws = _ws(L.mrinv_mc_workspace_size(n), dev)
    _check(L.mrinv_semi_markov_mc(_handle(dev), ctypes.byref(m), float(step), int(n), int(trajectories),
                                  ctypes.c_uint64(int(seed)), _ptr(A), _ptr(R), _ptr(tau), _ptr(jumps), _ptr(ws),
                                  ws.numel()))
    return (A, R, tau, jumps) if per_path else (A, R)


def residual_norms(q: torch.Tensor, X: torch.Tensor):
    """(sum_k ||e0 - A*X||_F, sum_k ||e0 - X*A||_F, max |e0 - A*X|) with A = e0 - q."""
    q = _square(q, "q")
    n, d, _ = q.shape
    X = _seq(X, "X", d, d, n=n)
    L = lib()
    ws = _ws(L.mrinv_workspace_size(8, d, n, 0, 0), q.device)
    out = (ctypes.c_double * 3)()
    _check(L.mrinv_residual_norms(_handle(q.device), _ptr(q), _ptr(X), d, n, out, _ptr(ws), ws.numel()))
    return float(out[0]), float(out[1]), float(out[2])


def psi_inverse_batched(qs, precision="mixed"):
    """Invert a list of kernels of uneven (d, n); returns the list of psi."""
    if not qs:
        return []
    qs = [_square(q, f"q[{i}]") for i, q in enumerate(qs)]
    dev = qs[0].device
    count = len(qs)
    prec = _PREC[precision]
    outs = [torch.empty_like(q) for q in qs]
    d_arr = (ctypes.c_int * count)(*[q.shape[1] for q in qs])
    n_arr = (ctypes.c_int64 * count)(*[q.shape[0] for q in qs])
    qp = (ctypes.c_void_p * count)(*[q.data_ptr() for q in qs])
    op = (ctypes.c_void_p * count)(*[o.data_ptr() for o in outs])
    L = lib()
    ws = _ws(L.mrinv_batched_workspace_size(_handle(dev), count, d_arr, n_arr, prec), dev)
    h = _handle(dev)
    _batched_owner[h.value] = None      # this call's plan replaces any prepared BatchedPlan on the stream
    _check(L.mrinv_psi_inverse_batched(h, count, qp, d_arr, n_arr, prec, op, _ptr(ws), ws.numel()))
    return outs


class BatchedPlan:
    """A prepared batched inversion (mrinv_psi_inverse_batched_prepare).

    The constructor plans every launch for the kernels ``qs`` and writes the
    descriptor table into its own workspace (it waits for the stream);
    :meth:`launch` only enqueues the launches, so it can be recorded into a
    CUDA/HIP graph on the same stream and replayed.  ``outs`` receive the
    inverses each time; ``qs`` must keep holding the inputs.  The library
    keeps one prepared plan per handle (per stream): preparing another plan on
    the same stream retires this one."""

    def __init__(self, qs, precision="mixed"):
        if not qs:
            raise MrinvError(1, "empty batch")
        self.qs = [_seq(q, f"q[{i}]") for i, q in enumerate(qs)]
        for i, q in enumerate(self.qs):
            if q.shape[1] != q.shape[2]:
                raise MrinvError(1, f"q[{i}] must be square")
        self.device = self.qs[0].device
        self.stream = torch.cuda.current_stream(self.device).cuda_stream
        count = len(self.qs)
        prec = _PREC[precision]
        self.outs = [torch.empty_like(q) for q in self.qs]
        d_arr = (ctypes.c_int * count)(*[q.shape[1] for q in self.qs])
        n_arr = (ctypes.c_int64 * count)(*[q.shape[0] for q in self.qs])
        qp = (ctypes.c_void_p * count)(*[q.data_ptr() for q in self.qs])
        op = (ctypes.c_void_p * count)(*[o.data_ptr() for o in self.outs])
        L = lib()
        self.h = _handle(self.device)
        self.ws = _ws(L.mrinv_batched_workspace_size(self.h, count, d_arr, n_arr, prec), self.device)
        _check(L.mrinv_psi_inverse_batched_prepare(self.h, count, qp, d_arr, n_arr, prec, op, _ptr(self.ws),
                                                   self.ws.numel()))
        _batched_owner[self.h.value] = id(self)

    def launch(self):
        if torch.cuda.current_stream(self.device).cuda_stream != self.stream:
            raise MrinvError(1, "launch on the stream the plan was prepared on")
        if _batched_owner.get(self.h.value) != id(self):
            raise MrinvError(1, "another batched plan was prepared on this stream since")
        _check(lib().mrinv_psi_inverse_batched_launch(self.h))
        return self.outs


_batched_owner: dict = {}


# ---------------------------------------------------------------------------
# Adjoint entry points
# ---------------------------------------------------------------------------

def _square(x: torch.Tensor, name: str) -> torch.Tensor:
    x = _seq(x, name)
    if x.shape[1] != x.shape[2]:
        raise MrinvError(1, f"{name} must be square, got {tuple(x.shape)}")
    return x


def psi_inverse_backward(psi: torch.Tensor, psi_bar: torch.Tensor) -> torch.Tensor:
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    psi_bar = _seq(psi_bar, "psi_bar", d, d, n=n)
    qb = torch.empty_like(psi)
    ws = _ws(lib().mrinv_workspace_size(3, d, n, 0, 0), psi.device)
    _check(lib().mrinv_psi_inverse_backward(_handle(psi.device), _ptr(psi), _ptr(psi_bar), d, n, _ptr(qb), _ptr(ws),
                                            ws.numel()))
    return qb


def markov_renewal_apply_backward(psi, L, M_bar, need_psi=True, need_L=True):
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    L = _seq(L, "L", rows=d, n=n)
    r = L.shape[2]
    M_bar = _seq(M_bar, "M_bar", d, r, n=n)
    pb = torch.zeros_like(psi) if need_psi else None
    lb = torch.empty_like(L) if need_L else None
    ws = _ws(lib().mrinv_workspace_size(4, d, n, r, 0), psi.device)
    _check(lib().mrinv_markov_renewal_apply_backward(_handle(psi.device), _ptr(psi), _ptr(L), _ptr(M_bar), d, n, r,
                                                     _ptr(pb), _ptr(lb), _ptr(ws), ws.numel()))
    return pb, lb


def transition_backward(psi, q, P_bar, need_psi=True, need_q=True):
    psi = _square(psi, "psi")
    n, d, _ = psi.shape
    q = _seq(q, "q", d, d, n=n)
    P_bar = _seq(P_bar, "P_bar", d, d, n=n)
    pb = torch.zeros_like(psi) if need_psi else None
    qb = torch.zeros_like(q) if need_q else None
    ws = _ws(lib().mrinv_workspace_size(5, d, n, 0, 0), psi.device)
    _check(lib().mrinv_transition_backward(_handle(psi.device), _ptr(psi), _ptr(q), _ptr(P_bar), d, n, _ptr(pb),
                                           _ptr(qb), _ptr(ws), ws.numel()))
    return pb, qb


def contract_backward(out_bar, rows, cols, u, v, cumulative=False, scale=1.0) -> torch.Tensor:
    if out_bar.device.type != "cuda" or out_bar.dtype != torch.float64 or out_bar.dim() != 1:
        raise MrinvError(1, "out_bar must be a 1-D float64 GPU tensor")
    out_bar = out_bar.contiguous()
    n = out_bar.numel()
    dev = out_bar.device
    Xb = torch.zeros((n, rows, cols), dtype=torch.float64, device=dev)
    u = _dvec(u, rows, dev)
    v = _dvec(v, cols, dev)
    _check(lib().mrinv_contract_backward(_handle(dev), _ptr(out_bar), n, rows, cols, _ptr(u), _ptr(v),
                                         int(cumulative), float(scale), _ptr(Xb)))
    return Xb


def scatter_block_add(Y_bar, rows, cols, rows_idx, cols_idx, X_bar=None) -> torch.Tensor:
    rows_idx = _indices(rows_idx, rows, "rows_idx", distinct=True)
    cols_idx = _indices(cols_idx, cols, "cols_idx", distinct=True)
    Y_bar = _seq(Y_bar, "Y_bar", rows_idx.numel(), cols_idx.numel())
    n = Y_bar.shape[0]
    dev = Y_bar.device
    if X_bar is None:
        X_bar = torch.zeros((n, rows, cols), dtype=torch.float64, device=dev)
    elif tuple(X_bar.shape) != (n, rows, cols) or not X_bar.is_contiguous() or X_bar.dtype != torch.float64:
        raise MrinvError(1, f"X_bar must be a contiguous float64 [{n}, {rows}, {cols}] tensor")
    ri = torch.as_tensor(rows_idx, dtype=torch.int32).to(dev).contiguous()
    ci = torch.as_tensor(cols_idx, dtype=torch.int32).to(dev).contiguous()
    _check(lib().mrinv_scatter_block_add(_handle(dev), _ptr(Y_bar), n, rows, cols, _ptr(ri), ri.numel(), _ptr(ci),
                                         ci.numel(), _ptr(X_bar)))
    return X_bar


# ---------------------------------------------------------------------------
# Autograd
# ---------------------------------------------------------------------------

class PsiInverse(torch.autograd.Function):
    """psi = (e0 - q)^-1 with the adjoint q_bar = Rev(psi^T * Rev(psi_bar) * psi^T)."""

    @staticmethod
    def forward(ctx, q, precision="fp64"):
        psi = psi_inverse(q, precision)
        ctx.save_for_backward(psi)
        return psi

    @staticmethod
    def backward(ctx, psi_bar):
        (psi,) = ctx.saved_tensors
        return psi_inverse_backward(psi, psi_bar.to(torch.float64)), None


class RenewalApply(torch.autograd.Function):
    """M = psi * L."""

    @staticmethod
    def forward(ctx, psi, L):
        ctx.save_for_backward(psi, L)
        return markov_renewal_apply(psi, L)

    @staticmethod
    def backward(ctx, M_bar):
        psi, L = ctx.saved_tensors
        pb, lb = markov_renewal_apply_backward(psi, L, M_bar, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return pb, lb


class Transition(torch.autograd.Function):
    """P = psi * Hbar(q)."""

    @staticmethod
    def forward(ctx, psi, q):
        ctx.save_for_backward(psi, q)
        return transition(psi, q)

    @staticmethod
    def backward(ctx, P_bar):
        psi, q = ctx.saved_tensors
        return transition_backward(psi, q, P_bar, ctx.needs_input_grad[0], ctx.needs_input_grad[1])


class Contract(torch.autograd.Function):
    """out(k) = offset + scale * u^T X(k) v (optionally cumulative); u, v constants."""

    @staticmethod
    def forward(ctx, X, u, v, cumulative=False, offset=0.0, scale=1.0):
        u = torch.as_tensor(u, dtype=torch.float64, device=X.device)
        v = torch.as_tensor(v, dtype=torch.float64, device=X.device)
        ctx.save_for_backward(u, v)
        ctx.meta = (X.shape[1], X.shape[2], bool(cumulative), float(scale))
        return contract(X, u, v, cumulative, offset, scale)

    @staticmethod
    def backward(ctx, ob):
        u, v = ctx.saved_tensors
        rows, cols, cum, scale = ctx.meta
        return contract_backward(ob.to(torch.float64), rows, cols, u, v, cum, scale), None, None, None, None, None


class GatherBlock(torch.autograd.Function):
    """Y(k) = X(k)[rows_idx, cols_idx]."""

    @staticmethod
    def forward(ctx, X, rows_idx, cols_idx):
        ctx.meta = (X.shape[1], X.shape[2], list(rows_idx), list(cols_idx))
        return gather_block(X, rows_idx, cols_idx)

    @staticmethod
    def backward(ctx, Yb):
        rows, cols, ri, ci = ctx.meta
        return scatter_block_add(Yb.to(torch.float64), rows, cols, ri, ci), None, None
