"""HIP path vs CPU oracle, element by element on the same seeded inputs (GPU only).

Tolerance: normwise relative 1e-5 for FP32 outputs, tangents, loss and gradients (the bound
the target states for complex64 arithmetic against the FP64 oracle); the FP64 plain path is
held to tighter bounds derived from its finite-difference step.
"""
import math
from copy import deepcopy

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


def _circuit(ctx, circ):
    from paper_2506_23246_amd.api import Circuit
    return Circuit(ctx, circ)


def _check_forward(ctx, circ, params, points, angles=None, jac=None, tol=TOL, name=""):
    c = _circuit(ctx, circ)
    out, tan = c.simulate(params, points, angles, jac)
    f, g = O.simulate(circ, params, points, angles, jac)
    e_f, e_g = rel(t2n(out), f), rel(t2n(tan), g)
    report(f"forward {name} n={circ.n} P={len(f)}", f=e_f, g=e_g)
    assert e_f < tol and e_g < tol
    return c


def _check_maxwell(ctx, w, tol=TOL, name=""):
    c = _circuit(ctx, w.circuit)
    r = c.maxwell(w.params, w.points, w.loss)
    f, g, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    errs = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [L]),
                grad=rel(t2n(r["grad"]), grad))
    report(f"maxwell {name} n={w.circuit.n} P={len(w.points)}", **errs)
    for k, v in errs.items():
        assert v < tol, (k, v)
    return c, r


# ---------------------------------------------------------------- forward --------------------

@pytest.mark.parametrize("k,P", [(0, 300), (1, 257), (2, 129), (4, 9)])
def test_forward_configs(ctx, k, P):
    w = W.config(k, P=P)
    _check_forward(ctx, w.circuit, np.asarray(w.params, np.float32), np.asarray(w.points, np.float32),
                   name=W.CONFIG_NAMES[k])


@pytest.mark.parametrize("n", list(range(3, 13)))
def test_forward_every_qubit_count(ctx, n):
    """Random depth-2 circuits with mixed CNOT/CZ rings of several strides, every n the fused
    kernels support; P spans several tiles plus a ragged tail."""
    rng = np.random.default_rng(200 + n)
    rings = [W.ring(n, W.CNOT, 1) + W.ring(n, W.CZ, 2), W.ring(n, W.CZ, 1), W.ring(n, W.CNOT, 3)]
    circ = W.layered(n, 3, "xyz", lambda l: rings[l], out_qubits=[0, n - 1, n // 2])
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    ppw = max(1, (512 if n == 12 else 256) // (1 << (n - 3)))
    P = 3 * ppw + 1 if n < 12 else 5
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    _check_forward(ctx, circ, params, pts, name=f"random n={n}")


@pytest.mark.parametrize("outs", [[4], [8, 0, 3, 5, 1, 7, 2, 6]])
def test_output_count_extremes(ctx, outs):
    """The fewest (1) and the most (8) read-out qubits, in scrambled order: forward against the
    oracle, and with 8 outputs the whole Maxwell step (the first three outputs are the fields, the
    other five are read out only)."""
    from types import SimpleNamespace
    rng = np.random.default_rng(400 + len(outs))
    n = 9
    rings = [W.ring(n, W.CNOT, 1), W.ring(n, W.CZ, 2)]
    circ = W.layered(n, 2, "rot", lambda l: rings[l], out_qubits=list(outs))
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 2 * (256 // (1 << (n - 3))) + 3      # two whole tiles and a ragged one
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    _check_forward(ctx, circ, params, pts, name=f"m={len(outs)}")
    if len(outs) >= 3:
        w = SimpleNamespace(circuit=circ, params=params, points=pts,
                            loss=W.MaxwellDesc(W.LOSS_DIEL_INTUITIVE, eps_r=4.0, x_interface=0.2))
        _check_maxwell(ctx, w, name="m=8")


@pytest.mark.parametrize("case", ["rings5", "empty5", "rings8"])
def test_parameter_free_circuits(ctx, case):
    """Circuits with no trainable gate (K = 0: entangler rings only, or nothing after the
    encoding): the plan has one round of identity slots; outputs, tangents and the Maxwell loss
    against the oracle, and an empty gradient."""
    n, gates, outs = {"rings5": (5, W.ring(5, W.CNOT, 1) + W.ring(5, W.CZ, 2), [0, 1, 2]),
                      "empty5": (5, [], [0, 1, 2]),
                      "rings8": (8, W.ring(8, W.CZ, 1) + W.ring(8, W.CNOT, 3), [0, 4, 7])}[case]
    circ = W.Circuit(n=n, gates=gates, n_params=0, out_qubits=outs)
    params = np.zeros(0, np.float32)
    pts = np.random.default_rng(500 + n).uniform(-1, 1, (2 * (256 >> (n - 3)) + 3, 3)).astype(np.float32)
    c = _check_forward(ctx, circ, params, pts, name=f"K=0 {case}")
    loss = W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=0.1)
    r = c.maxwell(params, pts, loss)
    f, g, L, grad = O.maxwell_eval(circ, params, pts, loss)
    e = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [L]))
    report(f"maxwell K=0 {case} P={len(pts)}", **e)
    assert all(v < TOL for v in e.values()), e
    assert grad.size == 0 and t2n(r["grad"]).size == 0


@pytest.mark.parametrize("gate,scale", [(W.ENC_RX, W.SCALE_ACOS), (W.ENC_RX, W.SCALE_ASIN),
                                        (W.ENC_RY, W.SCALE_BIAS), (W.ENC_RY, W.SCALE_NONE),
                                        (W.ENC_RX, W.SCALE_PI)])
def test_forward_encodings(ctx, gate, scale):
    rng = np.random.default_rng(7)
    enc = W.Encoding(kind=W.ENC_CYCLE, gate=gate, scale=scale)
    circ = W.strongly_entangling(7, 3, "rot", ent=W.CNOT, enc=enc)
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    pts = rng.uniform(-0.95, 0.95, (70, 3)).astype(np.float32)
    _check_forward(ctx, circ, params, pts, name=f"enc gate={gate} scale={scale}")


def test_forward_angle_encoding(ctx):
    """Per-point angles and Jacobian given (the hybrid-layer interface), the paper's 7-qubit,
    4-layer basic-entangling shape."""
    rng = np.random.default_rng(8)
    circ = W.basic_entangling(7, 4, "rot", enc=W.Encoding(kind=W.ENC_ANGLES, gate=W.ENC_RX))
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 75
    ang = rng.uniform(0, math.pi, (P, 7)).astype(np.float32)
    jac = rng.standard_normal((P, 7, 3)).astype(np.float32)
    _check_forward(ctx, circ, params, None, ang, jac, name="angles")


def test_no_entanglement_bloch_closed_form_n12(ctx):
    """Product-state circuit at 12 qubits against the closed Bloch form (no oracle statevector)."""
    n = 12
    rng = np.random.default_rng(9)
    circ = W.no_entanglement(n, 2, "xyz")
    circ.out_qubits = [0, 5, 11]
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    pts = rng.uniform(-1, 1, (6, 3)).astype(np.float32)
    c = _circuit(ctx, circ)
    out, _ = c.simulate(params, pts)
    out = t2n(out)
    for j, q in enumerate(circ.out_qubits):
        th = math.pi * pts[:, q % 3].astype(np.float64)
        b = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], 1)
        for (k, qq, _, p) in circ.gates:
            if qq != q:
                continue
            a = float(params[p])
            cs, sn = math.cos(a), math.sin(a)
            R = {W.RX: [[1, 0, 0], [0, cs, -sn], [0, sn, cs]], W.RY: [[cs, 0, sn], [0, 1, 0], [-sn, 0, cs]],
                 W.RZ: [[cs, -sn, 0], [sn, cs, 0], [0, 0, 1]]}[k]
            b = b @ np.array(R).T
        assert np.abs(out[:, j] - b[:, 2]).max() < 2e-6


# ---------------------------------------------------------------- Maxwell --------------------

@pytest.mark.parametrize("k,P", [(1, 300), (2, 150), (4, 6)])
def test_maxwell_configs(ctx, k, P):
    _check_maxwell(ctx, W.config(k, P=P), name=W.CONFIG_NAMES[k])


@pytest.mark.parametrize("kind", [W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT, W.LOSS_DIEL_INTUITIVE])
def test_maxwell_loss_kinds(ctx, kind):
    w = W.config(1, P=200)
    w.loss = W.MaxwellDesc(kind, eps_r=4.0, x_interface=0.1)
    _check_maxwell(ctx, w, name=f"loss kind {kind}")


@pytest.mark.parametrize("x_if", [-2.0, 2.0])
def test_split_loss_with_an_empty_region(ctx, x_if):
    """Every point on one side of the interface: the empty region's mean contributes nothing (no
    division by its zero count), the other region is averaged over all points."""
    w = W.config(1, P=200)
    w.loss = W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=x_if)
    _check_maxwell(ctx, w, name=f"split, interface at x = {x_if}")


@pytest.mark.parametrize("n,layers", [(3, 1), (4, 3), (8, 3), (11, 2), (12, 2)])
def test_maxwell_both_exchange_shapes(ctx, n, layers):
    """Whole Maxwell step with the software-pipelined exchange (two plane pairs) and with the
    unpipelined one (one plane pair): both against the oracle, on mixed CNOT/CZ rings (sign and
    sign-free exchanges), single-round circuits included; P spans tiles plus a ragged tail."""
    from paper_2506_23246_amd.api import Circuit
    rng = np.random.default_rng(300 + n)
    rings = [W.ring(n, W.CNOT, 1) + W.ring(n, W.CZ, 2), W.ring(n, W.CZ, 1), W.ring(n, W.CNOT, 2)]
    circ = W.layered(n, layers, "xyz", lambda l: rings[l % 3] if layers > 1 else [],
                     out_qubits=[0, n - 1, n // 2])
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    ppw = max(1, (512 if n == 12 else 256) // (1 << (n - 3)))
    P = 2 * ppw + 1 if n < 12 else 3
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    loss = W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=0.0)
    f, g, L, grad = O.maxwell_eval(circ, params, pts, loss)
    res = {}
    for planes in (4, 2):
        c = Circuit(ctx, circ)
        c.set_launch(planes, 1)
        r = c.maxwell(params, pts, loss)
        errs = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [L]),
                    grad=rel(t2n(r["grad"]), grad))
        report(f"maxwell exchange planes={planes} n={n} L={layers} P={P}", **errs)
        for k, v in errs.items():
            assert v < TOL, (planes, k, v)
        res[planes] = t2n(r["grad"])
    assert rel(res[2], res[4]) < TOL


@pytest.mark.parametrize("case", range(7))
def test_opening_stage_fold(ctx, case):
    """Circuits that open with rotations (folded into the encoding, statistics at the stage output),
    with an entangler (nothing folded), with a partial or split opening stage, or without any
    entangler: forward, tangents, loss and gradient against the oracle, at a ragged point count."""
    from tests.circuit_cases import opening_stage_cases
    name, circ, nh = opening_stage_cases()[case]
    rng = np.random.default_rng(500 + case)
    w = W.Workload(name, circ, rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32),
                   rng.uniform(-1, 1, (37, 3)).astype(np.float32), W.MaxwellDesc(W.LOSS_VACUUM))
    c, _ = _check_maxwell(ctx, w, name=name)
    assert c.info(11) == nh
    _check_forward(ctx, circ, w.params, w.points, name=name)


@pytest.mark.parametrize("k,P", [(1, 3000), (2, 700), (4, 5)])
def test_autotuned_launch_keeps_parity(ctx, k, P):
    """QP_FLAG_TUNE times the legal launch shapes (exchange planes, workgroups per CU) on first use
    and keeps the fastest: the tuned step matches the oracle, the chosen shape is a legal one, and
    later untuned calls reuse it with bitwise-equal per-point results."""
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    w = W.config(k, P=P)
    c = Circuit(ctx, w.circuit)
    r = c.maxwell(w.params, w.points, w.loss, flags=L.QP_FLAG_TUNE)
    f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    errs = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [Lo]),
                grad=rel(t2n(r["grad"]), grad))
    report(f"tuned maxwell {w.name} exchange planes={c.info(8)} wg/CU={c.info(9)}", **errs)
    for key, v in errs.items():
        assert v < TOL, (key, v)
    assert c.info(8) in (2, 4) and 1 <= c.info(9) <= 4
    out0, tan0 = t2n(r["out"]).copy(), t2n(r["tan"]).copy()
    r2 = c.maxwell(w.params, w.points, w.loss)
    assert np.array_equal(t2n(r2["out"]), out0) and np.array_equal(t2n(r2["tan"]), tan0)


def test_maxwell_batch_circuits_individually(ctx):
    """Every circuit of the uneven batch through the single-circuit fused path (small P)."""
    for w in W.batch_config(P_cap=40)[:8]:
        _check_maxwell(ctx, w, name=w.name)


def test_vjp_matches_oracle_reverse_mode(ctx):
    rng = np.random.default_rng(11)
    w = W.config(2, P=90)
    c = _circuit(ctx, w.circuit)
    d_out = rng.standard_normal((90, 3)).astype(np.float32)
    d_tan = rng.standard_normal((90, 3, 3)).astype(np.float32)
    got = t2n(c.vjp(w.params, w.points, d_out, d_tan))
    exp = O.grad_reverse(w.circuit, w.params, w.points, d_out, d_tan)
    e = rel(got, exp)
    report("vjp c3", grad=e)
    assert e < TOL


def test_structural_zero_gradients(ctx):
    """Last-layer RZ gradients vanish exactly in exact arithmetic; in FP32 they stay at noise."""
    w = W.config(1, P=128)
    c = _circuit(ctx, w.circuit)
    g = t2n(c.maxwell(w.params, w.points, w.loss)["grad"])
    n = 6
    last = [w.circuit.n_params - 3 * n + 3 * q + 2 for q in range(n)]
    assert np.abs(g[last]).max() < 1e-5 * np.abs(g).max()


def test_autograd_function(ctx):
    import torch
    from paper_2506_23246_amd.autograd import qcircuit
    rng = np.random.default_rng(12)
    w = W.config(1, P=64)
    c = _circuit(ctx, w.circuit)
    prm = torch.tensor(w.params, device="cuda", requires_grad=True)
    pts = torch.tensor(w.points, device="cuda")
    A = torch.tensor(rng.standard_normal((64, 3)), device="cuda", dtype=torch.float32)
    B = torch.tensor(rng.standard_normal((64, 3, 3)), device="cuda", dtype=torch.float32)
    out, tan = qcircuit(prm, pts, c)
    (out * A).sum().add((tan * B).sum()).backward()
    exp = O.grad_reverse(w.circuit, w.params, w.points, t2n(A), t2n(B))
    e = rel(t2n(prm.grad), exp)
    report("autograd", grad=e)
    assert e < TOL


def test_determinism_bitwise(ctx):
    w = W.config(2, P=500)
    c = _circuit(ctx, w.circuit)
    r1 = {k: t2n(v).copy() for k, v in c.maxwell(w.params, w.points, w.loss).items()}
    r2 = {k: t2n(v).copy() for k, v in c.maxwell(w.params, w.points, w.loss).items()}
    for k in r1:
        assert np.array_equal(r1[k], r2[k]), k


def test_empty_batch_of_points(ctx):
    w = W.config(1, P=0)
    w.points = np.zeros((0, 3), np.float32)
    c = _circuit(ctx, w.circuit)
    r = c.maxwell(w.params, w.points, w.loss)
    assert t2n(r["loss"])[0] == 0.0
    assert np.all(t2n(r["grad"]) == 0.0)


# ---------------------------------------------------------------- plain ----------------------

def test_plain_fp64_c1_forward_and_fd_tangents(ctx):
    w = W.config(0)
    c = _circuit(ctx, w.circuit)
    out, tan = c.plain_eval(w.params, w.points, precision=64, h=1e-5)
    f, g = O.simulate(w.circuit, w.params, w.points)
    fd = O.fd_tangents(w.circuit, w.params, w.points, h=1e-5)
    e = dict(f=rel(t2n(out), f), g_vs_analytic=rel(t2n(tan), g), g_vs_oracle_fd=rel(t2n(tan), fd))
    report("plain fp64 c1", **e)
    assert e["f"] < 1e-12 and e["g_vs_oracle_fd"] < 1e-9 and e["g_vs_analytic"] < 1e-8


def test_plain_fp32_forward(ctx):
    w = W.config(1, P=100)
    c = _circuit(ctx, w.circuit)
    out, tan = c.plain_eval(w.params, w.points, precision=32)
    f, g = O.simulate(w.circuit, w.params, w.points)
    e = dict(f=rel(t2n(out), f), g=rel(t2n(tan), g))
    report("plain fp32", **e)
    assert e["f"] < TOL and e["g"] < 2e-3


def test_plain_fp64_maxwell_fd_gradients(ctx):
    w = W.config(1, P=64)
    c = _circuit(ctx, w.circuit)
    ks = [0, 1, 40, 89]
    lo, dp = c.plain_maxwell_fd(w.params.astype(np.float64), w.points.astype(np.float64), w.loss, precision=64,
                                h=1e-5, h_param=1e-5, k_begin=0, k_end=2)
    _, _, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    dp = t2n(dp)
    assert abs(t2n(lo)[0] - L) < 1e-8 * max(1, abs(L))
    assert np.abs(dp[:2] - grad[:2]).max() < 1e-5 * max(1, np.abs(grad).max())
    del ks
