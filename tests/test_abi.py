"""The C-ABI library loads and exports every symbol include/qpinn.h declares (CPU only: no
compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpinn.h")
LIB = os.path.join(ROOT, "paper_2506_23246_amd", "libqpinn.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qp_simulate", "qp_vjp", "qp_maxwell_fused", "qp_batch_run", "qp_plain_eval",
                     "qp_circuit_compile", "qp_workspace_bytes", "qp_ctx_create", "qp_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    h = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(h, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2506_23246_amd import _lib
    assert sorted(_lib.SYMBOLS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_path_without_device_is_a_status_code():
    """With no usable GPU, creating a context must fail with a status, not crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present; covered by tests/test_gpu_errors.py")
    from paper_2506_23246_amd import _lib
    h = ctypes.c_void_p()
    st = _lib.qp_ctx_create(0, None, ctypes.byref(h))
    assert st in (_lib.QP_EDEVICE, _lib.QP_EINVAL)
