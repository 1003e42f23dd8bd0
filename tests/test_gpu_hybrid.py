"""Input gradients of the angle-given encoding (dL/d angles, dL/d Jacobian) and the hybrid
QPINN model on the GPU, against the CPU oracle.

The paper's hybrid model feeds the circuit per-point angles from a classical network (section
"QPINN architecture and ansatz designs": 7 qubits, 4 layers, RX angle embedding of tanh
activations with one of the five scalings of eq. scale).  The engine's adjoint returns, besides
the parameter gradient, the gradients with respect to those angles and their Jacobian, so that
torch can carry them into the network.  Normwise relative error per quantity, bar 1e-5.
"""
import math

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


def _scaled(kind, a, da):
    """theta = scale(a) and J = scale'(a) da for activations a in (-1, 1) (eq. scale)."""
    a = a.astype(np.float64)
    if kind == W.SCALE_NONE:
        th, d = a, np.ones_like(a)
    elif kind == W.SCALE_PI:
        th, d = math.pi * a, np.full_like(a, math.pi)
    elif kind == W.SCALE_BIAS:
        th, d = (a + 1) * math.pi / 2, np.full_like(a, math.pi / 2)
    elif kind == W.SCALE_ASIN:
        th, d = np.arcsin(a) + math.pi / 2, 1 / np.sqrt(1 - a * a)
    else:
        th, d = np.arccos(a), -1 / np.sqrt(1 - a * a)
    return th.astype(np.float32), (d[:, :, None] * da).astype(np.float32)


def _inputs(n, P, seed, scale=W.SCALE_ACOS):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.95, 0.95, (P, n))
    da = rng.standard_normal((P, n, 3))
    th, J = _scaled(scale, a, da)
    return th, J, rng


def _circuit(kind, n, L, gate=W.ENC_RX):
    enc = W.Encoding(kind=W.ENC_ANGLES, gate=gate)
    if kind == "basic":
        c = W.basic_entangling(n, L, "rot", enc=enc)
    elif kind == "strong_cz":
        c = W.strongly_entangling(n, L, "rot", ent=W.CZ, enc=enc)
    elif kind == "noent":
        c = W.no_entanglement(n, L, "xyz", enc=enc)
    elif kind == "ring_first":     # an entangler before any rotation: no opening stage to fold
        c = W.layered(n, L, "xyz", lambda l: W.ring(n, W.CNOT, 1), enc=enc)
        c.gates = W.ring(n, W.CZ, 1) + W.ring(n, W.CNOT, 1) + c.gates
    else:
        raise ValueError(kind)
    c.out_qubits = list(range(min(n, 8)))
    return c


def _check_vjp(ctx, circ, th, J, rng, P, label, planes=None):
    from paper_2506_23246_amd.api import Circuit
    prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    m = len(circ.out_qubits)
    sf = rng.standard_normal((P, m)).astype(np.float32)
    sg = rng.standard_normal((P, m, 3)).astype(np.float32)
    c = Circuit(ctx, circ)
    if planes:
        c.set_launch(planes, 1)
    g, ga, gj = c.vjp(prm, None, sf, sg, angles=th, jac=J, input_grads=True)
    ref_g, ref_a, ref_j = O.grad_reverse(circ, prm, None, sf.astype(np.float64), sg.astype(np.float64), th, J,
                                         inputs=True)
    errs = dict(params=rel(t2n(g), ref_g), angles=rel(t2n(ga), ref_a), jac=rel(t2n(gj), ref_j))
    report(f"input grads {label}", **errs)
    assert all(v < TOL for v in errs.values()), errs
    # the parameter gradient alone (no input gradients requested) is unchanged
    g2 = c.vjp(prm, None, sf, sg, angles=th, jac=J)
    assert rel(t2n(g2), ref_g) < TOL


@pytest.mark.parametrize("scale", [W.SCALE_NONE, W.SCALE_PI, W.SCALE_BIAS, W.SCALE_ASIN, W.SCALE_ACOS])
def test_paper_shape_vjp_input_grads_every_scaling(ctx, scale):
    circ = _circuit("basic", 7, 4)
    th, J, rng = _inputs(7, 40, 10 + scale, scale)
    _check_vjp(ctx, circ, th, J, rng, 40, f"7q4L basic RX scale {W.SCALE_NAMES[scale]}")


@pytest.mark.parametrize("kind,n,L,gate,P", [
    ("basic", 3, 2, W.ENC_RY, 50),        # one thread per point (register bits only)
    ("strong_cz", 7, 4, W.ENC_RX, 40),
    ("noent", 5, 3, W.ENC_RY, 40),
    ("ring_first", 6, 2, W.ENC_RX, 40),   # no opening rotation stage
    ("basic", 8, 3, W.ENC_RX, 24),        # swap slots
    ("basic", 10, 2, W.ENC_RY, 8),        # a point spans two waves
    ("basic", 12, 2, W.ENC_RX, 4),        # a point spans eight waves
])
def test_vjp_input_grads_shapes(ctx, kind, n, L, gate, P):
    circ = _circuit(kind, n, L, gate)
    th, J, rng = _inputs(n, P, 100 + n)
    _check_vjp(ctx, circ, th, J, rng, P, f"{kind} {n}q{L}L gate {gate}")


def test_vjp_input_grads_one_plane_pair(ctx):
    circ = _circuit("basic", 7, 4)
    th, J, rng = _inputs(7, 40, 77)
    _check_vjp(ctx, circ, th, J, rng, 40, "7q4L, unpipelined exchanges", planes=2)


@pytest.mark.parametrize("loss_kind", [W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT])
def test_maxwell_input_grads(ctx, loss_kind):
    from paper_2506_23246_amd.api import Circuit
    circ = _circuit("basic", 7, 4)
    P = 48
    th, J, rng = _inputs(7, P, 5)
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    desc = W.MaxwellDesc(loss_kind)
    c = Circuit(ctx, circ)
    r = c.maxwell(prm, pts, desc, angles=th, jac=J, input_grads=True)
    f, g = O.simulate(circ, prm, pts, th, J)
    L = O.maxwell_loss(g, pts, desc)
    ref_g, ref_a, ref_j = O.grad_reverse(circ, prm, pts, None, O.maxwell_seeds(g, pts, desc), th, J, inputs=True)
    errs = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [L]),
                params=rel(t2n(r["grad"]), ref_g), angles=rel(t2n(r["d_angles"]), ref_a),
                jac=rel(t2n(r["d_jac"]), ref_j))
    report(f"maxwell input grads loss {loss_kind}", **errs)
    assert all(v < TOL for v in errs.values()), errs


def test_input_grads_many_tiles_sampled(ctx):
    """Per-point input gradients do not depend on how points are grouped into tiles: at a size
    where every workgroup runs several tiles, sampled points match the oracle evaluated on those
    points alone."""
    from paper_2506_23246_amd.api import Circuit
    circ = _circuit("basic", 7, 4)
    P = 3 * 512 * 16 + 11
    th, J, rng = _inputs(7, P, 31)
    prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    sf = rng.standard_normal((P, 7)).astype(np.float32)
    sg = rng.standard_normal((P, 7, 3)).astype(np.float32)
    c = Circuit(ctx, circ)
    _, ga, gj = c.vjp(prm, None, sf, sg, angles=th, jac=J, input_grads=True)
    idx = np.unique(np.r_[np.linspace(0, P - 1, 12).astype(int), [P - 2]])
    _, ref_a, ref_j = O.grad_reverse(circ, prm, None, sf[idx].astype(np.float64), sg[idx].astype(np.float64),
                                     th[idx], J[idx], inputs=True)
    errs = dict(angles=rel(t2n(ga)[idx], ref_a), jac=rel(t2n(gj)[idx], ref_j))
    report(f"input grads sampled P={P}", **errs)
    assert all(v < TOL for v in errs.values()), errs


def test_input_grads_need_the_angle_encoding(ctx):
    import torch
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    w = W.config(1, P=16)
    c = Circuit(ctx, w.circuit)
    with pytest.raises(L.QPError) as e:
        c.vjp(w.params, w.points, np.zeros((16, 3), np.float32), input_grads=True)
    assert e.value.status == L.QP_EINVAL
    circ = _circuit("basic", 7, 2)
    th, J, rng = _inputs(7, 16, 1)
    c2 = Circuit(ctx, circ)
    with pytest.raises(L.QPError) as e:
        c2.vjp(rng.uniform(0, 6, circ.n_params).astype(np.float32), None, np.zeros((16, 7), np.float32),
               angles=th, jac=J, input_grads=True, flags=L.QP_FLAG_DENSE_MFMA)
    assert e.value.status == L.QP_EUNSUPPORTED
    torch.cuda.synchronize()


def test_hybrid_model_end_to_end_gradients(ctx):
    """The paper's hybrid model (RFF, 256- and 128-neuron tanh layers, 7 tanh activations scaled by
    acos, the 7-qubit 4-layer circuit with RX embedding, Linear(7, 3) head) on the GPU: loss and
    every parameter gradient (network weights, circuit parameters, head) against the same model
    in float64 on the CPU with the oracle in place of the engine."""
    import torch
    from paper_2506_23246_amd.hybrid import HybridQPINN, maxwell_residual_loss
    from tests.hybrid_reference import oracle_circuit_fn
    circ = W.paper_context_circuit("basic")
    P = 64
    pts = np.random.default_rng(3).uniform(-1, 1, (P, 3)).astype(np.float32)
    gpu = HybridQPINN(circ, ctx=ctx, seed=4).cuda()
    ref = HybridQPINN(circ, circuit_fn=oracle_circuit_fn(circ), seed=4, dtype=torch.float64)
    with torch.no_grad():
        for (n1, p1), (n2, p2) in zip(gpu.named_parameters(), ref.named_parameters()):
            assert n1 == n2
            p2.copy_(p1.detach().cpu().double())
        ref.B.copy_(gpu.B.detach().cpu().double())
    x = torch.tensor(pts, device="cuda")
    fields, dfields = gpu(x)
    loss = maxwell_residual_loss(dfields, x)
    loss.backward()
    xr = torch.tensor(pts, dtype=torch.float64)
    rf, rdf = ref(xr)
    rloss = maxwell_residual_loss(rdf, xr)
    rloss.backward()
    errs = {"fields": rel(t2n(fields), rf.detach().numpy()), "dfields": rel(t2n(dfields), rdf.detach().numpy()),
            "loss": rel([float(loss.detach())], [float(rloss.detach())])}
    for (name, p1), (_, p2) in zip(gpu.named_parameters(), ref.named_parameters()):
        if p2.grad is not None:
            errs["grad " + name] = rel(t2n(p1.grad), p2.grad.numpy())
    report("hybrid model", **errs)
    assert all(v < TOL for v in errs.values()), errs
