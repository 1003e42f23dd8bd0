"""ctypes binding of libqpinn.so: the C ABI of include/qpinn.h under the same names.

Argument marshalling only - every step of the hot path runs in the library's HIP kernels.  The
library is loaded from this package directory; if it is missing, ``lib()`` raises (there is no
fallback of any kind).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpinn.so")

QP_OK, QP_EINVAL, QP_ESHAPE, QP_EUNSUPPORTED, QP_EWORKSPACE, QP_EDEVICE = range(6)
STATUS_NAMES = {0: "QP_OK", 1: "QP_EINVAL", 2: "QP_ESHAPE", 3: "QP_EUNSUPPORTED", 4: "QP_EWORKSPACE",
                5: "QP_EDEVICE"}
QP_FLAG_NO_TANGENTS, QP_FLAG_LOSS_SUM, QP_FLAG_TUNE, QP_FLAG_DENSE_MFMA, QP_FLAG_GATES_FP32 = 0x1, 0x2, 0x4, 0x8, 0x10


class qp_gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32), ("param", C.c_int32)]


class qp_encoding(C.Structure):
    _fields_ = [("kind", C.c_int32), ("gate", C.c_int32), ("scale", C.c_int32), ("n_features", C.c_int32),
                ("coord_of_qubit", C.POINTER(C.c_int32)), ("rff_B", C.POINTER(C.c_float)),
                ("rff_W", C.POINTER(C.c_float))]


class qp_circuit_desc(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_params", C.c_int32), ("n_gates", C.c_int32),
                ("gates", C.POINTER(qp_gate)), ("enc", qp_encoding), ("n_out", C.c_int32),
                ("out_qubits", C.POINTER(C.c_int32))]


class qp_maxwell_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("eps_r", C.c_float), ("x_interface", C.c_float)]


class qp_total_loss_desc(C.Structure):
    _fields_ = [("phys", qp_maxwell_desc), ("w_ic", C.c_float), ("w_sym", C.c_float), ("w_energy", C.c_float),
                ("ic_a", C.c_float)]


class qp_batch_io(C.Structure):
    _fields_ = [("params", C.c_void_p), ("points", C.c_void_p), ("out", C.c_void_p), ("tan", C.c_void_p),
                ("loss", C.c_void_p), ("d_params", C.c_void_p)]


# name -> (restype, argtypes); every symbol declared in include/qpinn.h
_P = C.c_void_p
_SIGS = {
    "qp_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "qp_ctx_set_stream": (C.c_int, [_P, _P]),
    "qp_ctx_destroy": (None, [_P]),
    "qp_last_error": (C.c_char_p, [_P]),
    "qp_sync": (C.c_int, [_P]),
    "qp_device_cu_count": (C.c_int32, [_P]),
    "qp_ctx_enable_kernel_timing": (C.c_int, [_P, C.c_int32]),
    "qp_ctx_last_kernel_ms": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "qp_circuit_compile": (C.c_int, [_P, C.POINTER(qp_circuit_desc), C.POINTER(_P)]),
    "qp_circuit_destroy": (None, [_P]),
    "qp_circuit_info": (C.c_int64, [_P, C.c_int32]),
    "qp_circuit_set_launch": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "qp_circuit_set_dense_chunk": (C.c_int, [_P, C.c_int32]),
    "qp_plan_image": (C.c_int, [C.POINTER(qp_circuit_desc), _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "qp_workspace_bytes": (C.c_size_t, [_P, C.c_int64, C.c_uint32]),
    "qp_simulate": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int64, _P, _P, _P, C.c_size_t, C.c_uint32]),
    "qp_vjp": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int64, _P, _P, _P, _P, _P, _P, C.c_size_t, C.c_uint32]),
    "qp_maxwell_fused": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int64, C.POINTER(qp_maxwell_desc), _P, _P, _P,
                                   _P, _P, _P, _P, C.c_size_t, C.c_uint32]),
    "qp_total_workspace_bytes": (C.c_size_t, [_P, C.c_int64, C.c_int64, C.c_int32]),
    "qp_total_loss": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, C.c_int64, C.POINTER(qp_total_loss_desc), _P, _P,
                                _P, _P, _P, C.c_size_t, C.c_uint32]),
    "qp_bloch": (C.c_int, [_P, _P, C.c_int32, _P, _P, _P, C.c_int64, _P, _P, _P, C.c_size_t]),
    "qp_energy_workspace_bytes": (C.c_size_t, [_P, C.c_int64, C.c_int64, C.c_int64]),
    "qp_energy_profile": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, C.c_int64, _P, C.c_int64,
                                    C.POINTER(qp_maxwell_desc), _P, _P, C.c_size_t, C.c_uint32]),
    "qp_noalloc_scratch_bytes": (C.c_size_t, []),
    "qp_maxwell_fused_noalloc": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int64, C.POINTER(qp_maxwell_desc), _P, _P,
                                           _P, _P, _P, _P, C.c_uint32]),
    "qp_batch_compile": (C.c_int, [_P, C.c_int32, C.POINTER(qp_circuit_desc), C.POINTER(C.c_int64),
                                   C.POINTER(_P)]),
    "qp_batch_destroy": (None, [_P]),
    "qp_batch_workspace_bytes": (C.c_size_t, [_P]),
    "qp_batch_run": (C.c_int, [_P, _P, C.POINTER(qp_batch_io), C.POINTER(qp_maxwell_desc), _P, C.c_size_t,
                               C.c_uint32]),
    "qp_batch_graph_launch": (C.c_int, [_P, _P, C.POINTER(qp_batch_io), C.POINTER(qp_maxwell_desc), _P,
                                        C.c_size_t, C.c_uint32]),
    "qp_batch_info": (C.c_int64, [_P, C.c_int32]),
    "qp_plain_workspace_bytes": (C.c_size_t, [_P, C.c_int64, C.c_int32]),
    "qp_plain_eval": (C.c_int, [_P, _P, C.c_int32, _P, _P, C.c_int64, C.c_double, _P, _P, _P, C.c_size_t]),
    "qp_plain_maxwell_fd": (C.c_int, [_P, _P, C.c_int32, _P, _P, C.c_int64, C.POINTER(qp_maxwell_desc),
                                      C.c_double, C.c_double, C.c_int32, C.c_int32, _P, _P, _P, C.c_size_t]),
}
SYMBOLS = tuple(_SIGS)

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_23246_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


class QPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None):
    if status != QP_OK:
        msg = lib().qp_last_error(ctx).decode() if ctx else ""
        raise QPError(status, msg)


# thin wrappers with the C names (pointers are ints or None)
def _wrap(name):
    def f(*args):
        return getattr(lib(), name)(*args)
    f.__name__ = name
    return f


for _n in _SIGS:
    globals()[_n] = _wrap(_n)
