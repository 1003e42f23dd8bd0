"""Host logic: the planner rejects malformed circuit descriptors with the documented status codes
(no device needed: qp_plan_image runs the planner on the host only)."""
import ctypes as C
import os

import numpy as np
import pytest

import workloads as W

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2506_23246_amd",
                   "libqpinn.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _status(circ, with_buffer=True):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import make_desc
    d, keep = make_desc(circ)
    nb = C.c_size_t(0)
    st = L.qp_plan_image(C.byref(d), None, 0, C.byref(nb))
    if st == L.QP_EWORKSPACE and with_buffer:
        buf = (C.c_ubyte * nb.value)()
        st = L.qp_plan_image(C.byref(d), buf, nb.value, C.byref(nb))
    return st, nb.value


def _circ(n, gates, K, out=(0, 1, 2)):
    return W.Circuit(n=n, gates=list(gates), n_params=K, out_qubits=list(out))


def test_valid_plan_and_buffer_size_query():
    from paper_2506_23246_amd import _lib as L
    circ = W.config(1, P=1).circuit
    st, nb = _status(circ, with_buffer=False)
    assert st == L.QP_EWORKSPACE and nb > 0        # size query: no buffer given
    st, nb2 = _status(circ)
    assert st == L.QP_OK and nb2 == nb


@pytest.mark.parametrize("case", ["n0", "n15", "qubit", "cnot_same", "param", "kind", "n_out0", "out_qubit"])
def test_malformed_descriptors_are_status_codes(case):
    from paper_2506_23246_amd import _lib as L
    ok = [(W.RX, 0, -1, 0), (W.CNOT, 0, 1, -1)]
    circ, want = {
        "n0": (_circ(0, [], 0, out=()), (L.QP_EUNSUPPORTED, L.QP_ESHAPE)),
        "n15": (_circ(15, ok, 1), (L.QP_EUNSUPPORTED,)),
        "qubit": (_circ(4, [(W.RX, 4, -1, 0)], 1), (L.QP_EINVAL,)),
        "cnot_same": (_circ(4, [(W.CNOT, 2, 2, -1)], 0), (L.QP_EINVAL,)),
        "param": (_circ(4, [(W.RY, 1, -1, 3)], 2), (L.QP_EINVAL,)),
        "kind": (_circ(4, [(99, 1, -1, 0)], 1), (L.QP_EINVAL,)),
        "n_out0": (_circ(4, ok, 1, out=()), (L.QP_ESHAPE,)),
        "out_qubit": (_circ(4, ok, 1, out=(0, 7, 1)), (L.QP_EINVAL,)),
    }[case]
    st, _ = _status(circ)
    assert st in want, (case, st)


def test_plain_only_circuits_have_no_fused_plan():
    """13 qubits, and a CNOT after a CRZ within one entangler stage (the phase would have to move
    through the index map), are evaluated by the plain path only: the fused planner reports
    QP_EUNSUPPORTED instead of building register rounds.  A CRZ run alone plans."""
    from paper_2506_23246_amd import _lib as L
    st, _ = _status(W.layered(13, 1, "xyz", lambda l: W.ring(13, W.CNOT, 1)))
    assert st == L.QP_EUNSUPPORTED
    st, _ = _status(_circ(4, [(W.RX, 0, -1, 0), (W.CRZ, 0, 1, 1), (W.CNOT, 1, 2, -1), (W.RY, 2, -1, 2)], 3))
    assert st == L.QP_EUNSUPPORTED
    st, _ = _status(_circ(4, [(W.RX, 0, -1, 0), (W.CNOT, 1, 2, -1), (W.CRZ, 0, 1, 1), (W.RY, 2, -1, 2)], 3))
    assert st == L.QP_OK


def test_cross_mesh_phase_stages_in_the_plan_image():
    """The 7-qubit, 4-layer Cross-Mesh plan: one phase stage per layer but the last (a diagonal
    right before the Z readout changes no output and has zero gradient), n + n(n-1)/2 = 28
    coefficients and moments per stage, each CRZ parameter of the first three layers mapped to
    exactly one phase gate, the last layer's to none."""
    import ctypes as C
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import make_desc
    from tests.plan_emulator import HDR
    circ = W.paper_context_circuit("cross_mesh")
    d, keep = make_desc(circ)
    nb = C.c_size_t(0)
    L.qp_plan_image(C.byref(d), None, 0, C.byref(nb))
    buf = (C.c_ubyte * nb.value)()
    assert L.qp_plan_image(C.byref(d), buf, nb.value, C.byref(nb)) == L.QP_OK
    raw = bytes(buf)
    base = HDR.itemsize
    n_phase, off_phase, off_gates, n_coef, n_mom, off_ptr, off_idx = np.frombuffer(raw, "<i4", 7, base)
    assert n_phase == 3 and n_coef == n_mom == 3 * 28
    stages = np.frombuffer(raw, "<i4", 4 * 3, off_phase).reshape(3, 4)
    assert list(stages[:, 1]) == [42, 42, 42] and list(stages[:, 2]) == [0, 28, 56]
    ptr = np.frombuffer(raw, "<i4", circ.n_params + 1, off_ptr)
    crz = [p for (k, q0, q1, p) in circ.gates if k == W.CRZ]
    counts = np.diff(ptr)
    assert all(counts[p] == 1 for p in crz[:126]) and all(counts[p] == 0 for p in crz[126:])
