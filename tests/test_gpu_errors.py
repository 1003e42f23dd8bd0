"""Error paths of the C ABI on a GPU: every malformed call returns a status code with a message,
before any kernel is launched, and the context keeps working afterwards (GPU only; no case here
launches a kernel on bad arguments)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.gpu_helpers import TOL, rel, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_23246_amd.api import Context
    assert torch.cuda.is_available()
    return Context(0)


def _call(ctx, c, prm, pts, P, md, bufs, wp, nb, flags=0):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import _ptr
    return L.qp_maxwell_fused(ctx.h, c.h, _ptr(prm), _ptr(pts), None, None, P, C.byref(md) if md is not None else None,
                              _ptr(bufs["out"]), _ptr(bufs["tan"]), _ptr(bufs["loss"]), _ptr(bufs["grad"]), None, None,
                              wp, nb, flags)


def _setup(ctx, k=1, P=64):
    import torch
    from paper_2506_23246_amd.api import Circuit
    w = W.config(k, P=P)
    c = Circuit(ctx, w.circuit)
    dev = ctx.dev
    prm = torch.tensor(w.params, device=dev)
    pts = torch.tensor(w.points, device=dev)
    bufs = {"out": torch.empty((P, 3), device=dev), "tan": torch.empty((P, 3, 3), device=dev),
            "loss": torch.empty(1, dtype=torch.float64, device=dev), "grad": torch.empty(w.circuit.n_params, device=dev)}
    return w, c, prm, pts, bufs


def test_bad_calls_return_status_codes(env):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import maxwell_desc
    ctx = env
    w, c, prm, pts, bufs = _setup(ctx)
    P = len(w.points)
    _, wp, nb = c.workspace(P)
    md = maxwell_desc(w.loss)
    cases = {
        "workspace too small": (dict(nb=16), L.QP_EWORKSPACE),
        "workspace misaligned": (dict(wp=wp + 8), L.QP_EWORKSPACE),
        "P < 0": (dict(P=-1), L.QP_EINVAL),
        "P above 2^31 - 1": (dict(P=1 << 31), L.QP_EUNSUPPORTED),
        "params null": (dict(prm=None), L.QP_EINVAL),
        "loss descriptor null": (dict(md=None), L.QP_EINVAL),
    }
    for name, (over, want) in cases.items():
        a = dict(prm=prm, pts=pts, P=P, md=md, wp=wp, nb=nb)
        a.update(over)
        st = _call(ctx, c, a["prm"], a["pts"], a["P"], a["md"], bufs, a["wp"], a["nb"])
        assert st == want, (name, st)
        assert L.qp_last_error(ctx.h).decode(), name      # a message names the problem
    bad_kind = maxwell_desc(w.loss)
    bad_kind.kind = 7
    assert _call(ctx, c, prm, pts, P, bad_kind, bufs, wp, nb) == L.QP_EINVAL
    with pytest.raises(L.QPError):
        c.set_launch(3, 1)                                  # exchange planes must be 2 or 4
    # the context and circuit still work, and match the oracle
    r = c.maxwell(w.params, w.points, w.loss)
    f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    assert rel(t2n(r["out"]), f) < TOL and rel(t2n(r["grad"]), grad) < TOL


def test_unsupported_circuits(env):
    """A 13-qubit circuit compiles (the plain path runs it) but the fused step reports
    QP_EUNSUPPORTED; the Maxwell loss needs the three outputs (E_z, H_x, H_y): QP_ESHAPE."""
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    ctx = env
    big = W.layered(13, 1, "xyz", lambda l: W.ring(13, W.CNOT, 1))
    c = Circuit(ctx, big)
    rng = np.random.default_rng(1)
    with pytest.raises(L.QPError) as e:
        c.maxwell(rng.uniform(0, 6, big.n_params).astype(np.float32), rng.uniform(-1, 1, (4, 3)).astype(np.float32),
                  W.MaxwellDesc())
    assert e.value.status == L.QP_EUNSUPPORTED
    two = W.layered(4, 1, "xyz", lambda l: W.ring(4, W.CNOT, 1), out_qubits=[0, 1])
    c2 = Circuit(ctx, two)
    with pytest.raises(L.QPError) as e:
        c2.maxwell(rng.uniform(0, 6, two.n_params).astype(np.float32), rng.uniform(-1, 1, (4, 3)).astype(np.float32),
                   W.MaxwellDesc())
    assert e.value.status == L.QP_ESHAPE
