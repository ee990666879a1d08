"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and validates arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrinv.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mrinv_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2605_30379_amd as m
    if not os.path.exists(m.library_path):
        import __graft_entry__
        __graft_entry__.build()
    return m.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mrinv_psi_inverse", "mrinv_markov_renewal_apply", "mrinv_transition",
                 "mrinv_psi_inverse_batched", "mrinv_psi_inverse_backward",
                 "mrinv_markov_renewal_apply_backward"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_workspace_sizes(L):
    # op 0 = psi inverse
    assert L.mrinv_workspace_size(0, 4, 256, 0, 0) > 0
    assert L.mrinv_workspace_size(0, 65, 256, 0, 0) == 0
    assert L.mrinv_workspace_size(0, 4, 0, 0, 0) == 0
    # FP64 psi at d=16, n=65536: three packed spectra of 65536 rows x 128 lanes x 16 bytes,
    # plus outer-twiddle tables (at most 3 L entries of 16 bytes)
    spectra = 3 * 65536 * 128 * 16
    ws = L.mrinv_workspace_size(0, 16, 65536, 0, 0)
    assert spectra <= ws <= spectra + 3 * 65536 * 16 + 8192
    assert L.mrinv_workspace_size(0, 16, 65536, 0, 1) > L.mrinv_workspace_size(0, 16, 65536, 0, 0)
    # residual diagnostics (op 8): three float64 spectra at 2^ceil(log2(2n-1)) plus two copies of the input
    assert L.mrinv_workspace_size(8, 4, 100, 0, 0) >= 3 * 256 * 8 * 16 + 2 * 100 * 16 * 8


def test_argument_validation_without_gpu(L):
    # A NULL handle is rejected before any HIP call.
    st = L.mrinv_psi_inverse(None, None, 4, 16, 0, None, None, 0)
    assert st == 1
    assert b"NULL" in L.mrinv_last_error()
    assert L.mrinv_status_string(2) == b"A(0) singular"
    # The HBM probe checks its handle and pointers before any launch too.
    gbps = ctypes.c_double(-1.0)
    L.mrinv_hbm_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    assert L.mrinv_hbm_probe(None, None, 1 << 30, 0, 16, 3, ctypes.byref(gbps)) == 1
    assert gbps.value == -1.0


def test_product_path_has_no_cpu_fallback():
    """The binding refuses CPU tensors instead of computing on the host."""
    import torch
    import paper_2605_30379_amd as m
    with pytest.raises(m.MrinvError):
        m.psi_inverse(torch.zeros((4, 2, 2), dtype=torch.float64))


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2605_30379_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f), errors="replace").read()
                assert "import oracle" not in text and "from oracle" not in text and "liborc" not in text, f


def test_batched_workspace_query_without_a_handle(L):
    """The batched planner also sizes the workspace without a handle or GPU."""
    import ctypes
    import smk_inputs as si
    w = si.batch_workload()
    d = (ctypes.c_int * 512)(*[x["d"] for x in w])
    n = (ctypes.c_int64 * 512)(*[x["n"] for x in w])
    L.mrinv_batched_workspace_size.restype = ctypes.c_size_t
    fp64 = L.mrinv_batched_workspace_size(None, 512, d, n, 0)
    mixed = L.mrinv_batched_workspace_size(None, 512, d, n, 1)
    assert 0 < fp64 < mixed < (96 << 30)
    bad = (ctypes.c_int * 1)(65)
    one = (ctypes.c_int64 * 1)(10)
    assert L.mrinv_batched_workspace_size(None, 1, bad, one, 0) == 0
