"""qp_maxwell_fused_noalloc (scratch in the library's fixed device array) against
qp_maxwell_fused (caller workspace), through the C ABI, on two calls in a row with the second
one smaller; results must be bitwise equal (same kernels, same launch) and within the FP32 bar
of the oracle."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.gpu_helpers import TOL, rel, report, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_23246_amd.api import Context
    assert torch.cuda.is_available()
    return Context(0)


@pytest.mark.parametrize("k,sizes", [(1, (16384, 1000)), (2, (4096, 777)), (4, (300, 37))])
def test_noalloc_matches_workspace_entry_point(ctx, k, sizes):
    from paper_2506_23246_amd.api import Circuit
    w = W.config(k)
    c = Circuit(ctx, w.circuit)
    for P in sizes:
        pts = w.points[:P]
        a = c.maxwell(w.params, pts, w.loss)
        ref = {n: t2n(v).copy() for n, v in a.items()}
        b = c.maxwell_noalloc(w.params, pts, w.loss)
        got = {n: t2n(v) for n, v in b.items()}
        print(f"config {k} P={P}", flush=True)
        for n in ("out", "tan", "loss", "grad"):
            assert np.array_equal(got[n], ref[n]), n
        if P <= 1000 and k != 4:
            f, g, L, grad = O.maxwell_eval(w.circuit, w.params, pts, w.loss)
            errs = dict(f=rel(got["out"], f), g=rel(got["tan"], g), loss=rel(got["loss"], [L]),
                        grad=rel(got["grad"], grad))
            report(f"noalloc config {k} P={P}", **errs)
            assert all(v < TOL for v in errs.values()), errs


def test_noalloc_rejects_what_needs_a_workspace(ctx):
    import torch
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit, maxwell_desc
    cap = int(L.qp_noalloc_scratch_bytes())
    assert cap == 16 << 20
    w = W.config(2)                     # random Fourier features: scratch grows 16 n bytes per point
    c = Circuit(ctx, w.circuit)
    P = cap // (16 * w.circuit.n) + 4096
    assert int(L.qp_workspace_bytes(c.h, P, 0)) > cap
    dev = ctx.dev
    prm = torch.tensor(w.params, device=dev)
    pts = torch.zeros((P, 3), dtype=torch.float32, device=dev)
    out = torch.empty((P, 3), dtype=torch.float32, device=dev)
    tan = torch.empty((P, 3, 3), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(w.circuit.n_params, dtype=torch.float32, device=dev)
    md = maxwell_desc(w.loss)
    args = (ctx.h, c.h, prm.data_ptr(), pts.data_ptr(), None, None)
    tail = (C.byref(md), out.data_ptr(), tan.data_ptr(), loss.data_ptr(), grad.data_ptr(), None, None)
    st = L.qp_maxwell_fused_noalloc(*args, P, *tail, 0)
    assert st == L.QP_EWORKSPACE and b"scratch" in L.qp_last_error(ctx.h)
    for fl in (L.QP_FLAG_TUNE, L.QP_FLAG_DENSE_MFMA):
        assert L.qp_maxwell_fused_noalloc(*args, 64, *tail, fl) == L.QP_EUNSUPPORTED
    # the context still computes correctly afterwards
    r = c.maxwell_noalloc(w.params, w.points[:64], w.loss)
    f, g = O.simulate(w.circuit, w.params, w.points[:64])
    assert rel(t2n(r["out"]), f) < TOL and rel(t2n(r["tan"]), g) < TOL
