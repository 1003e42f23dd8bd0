"""The packed fused kernels (four points in the four statevector slots of a thread group, no input
tangents): outputs equal to those of the tangent-carrying kernel bit for bit (the same arithmetic
per statevector), at every qubit count with ragged last tiles, for the cycled, angle-given and
random-Fourier-feature encodings and for CRZ phase stages; the packed adjoint (output seeds only)
through the total loss against the oracle on several tiles."""
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


def _ppt(n):
    """Points per tile of the tangent-carrying kernel (512 threads at 12 qubits, else 256)."""
    return (512 if n == 12 else 256) // (1 << (n - 3))


@pytest.mark.parametrize("n", list(range(3, 13)))
def test_packed_forward_equals_tangent_kernel(ctx, n):
    from paper_2506_23246_amd.api import Circuit
    rng = np.random.default_rng(100 + n)
    circ = W.layered(n, 2, "xyz", lambda l: W.ring(n, W.CNOT if l == 0 else W.CZ, 1 + (l % 2)),
                     out_qubits=[n - 1, 0, n // 2])
    prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 4 * _ppt(n) * 3 + 5            # three packed tiles and a ragged one (one point in its last group)
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    c = Circuit(ctx, circ)
    f_tan, _ = c.simulate(prm, pts)
    f_pk, none = c.simulate(prm, pts, tangents=False)
    assert none is None
    assert np.array_equal(t2n(f_pk), t2n(f_tan))
    if n <= 8:
        f, _ = O.simulate(circ, prm, pts[:64])
        assert rel(t2n(f_pk)[:64], f) < TOL


def test_packed_forward_other_encodings_and_phases(ctx):
    from paper_2506_23246_amd.api import Circuit
    rng = np.random.default_rng(7)
    # angle-given encoding, the paper's 7-qubit shape
    circ = W.paper_context_circuit("basic")
    prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 157
    ang = rng.uniform(0, math.pi, (P, 7)).astype(np.float32)
    jac = rng.standard_normal((P, 7, 3)).astype(np.float32)
    c = Circuit(ctx, circ)
    a, _ = c.simulate(prm, None, ang, jac)
    b, _ = c.simulate(prm, None, ang, jac, tangents=False)
    assert np.array_equal(t2n(a), t2n(b))
    # random Fourier features (8 qubits) and Cross-Mesh CRZ phase stages (unpipelined kernel)
    for w in (W.config(2, P=203), None):
        if w is None:
            circ = W.cross_mesh(6, 3, "xz", W.CRZ)
            prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
            pts = rng.uniform(-1, 1, (301, 3)).astype(np.float32)
        else:
            circ, prm, pts = w.circuit, w.params, w.points
        c = Circuit(ctx, circ)
        a, _ = c.simulate(prm, pts)
        b, _ = c.simulate(prm, pts, tangents=False)
        assert np.array_equal(t2n(a), t2n(b)), circ.name
        f, _ = O.simulate(circ, prm, pts[:40])
        report(f"packed forward {circ.name}", f=rel(t2n(b)[:40], f))
        assert rel(t2n(b)[:40], f) < TOL


@pytest.mark.parametrize("case", ["c2_multitile", "cross_mesh"])
def test_packed_adjoint_through_the_total_loss(ctx, case):
    """Mirror and IC points (2P + P0 of them) go through the packed forward and adjoint: several
    packed tiles at 6 qubits, and a Cross-Mesh circuit whose phase stages run in the packed adjoint."""
    from paper_2506_23246_amd.api import Circuit
    rng = np.random.default_rng(11)
    if case == "c2_multitile":
        w = W.config(1, P=300)
        circ, prm, pts = w.circuit, w.params, w.points
        phys = w.loss
    else:
        circ = W.cross_mesh(5, 3, "x", W.CRZ)
        prm = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
        pts = rng.uniform(-1, 1, (45, 3)).astype(np.float32)
        phys = W.MaxwellDesc(W.LOSS_VACUUM)
    xy = W.ic_plane_points(rng, 50)
    desc = W.TotalLossDesc(phys=phys)
    c = Circuit(ctx, circ)
    r = c.total_loss(prm, pts, xy, desc)
    terms, grad = O.total_eval(circ, prm, pts, xy, desc)
    got = t2n(r["terms"])
    ref = np.array([terms["total"], terms["phys"], terms["ic"], terms["sym"], terms["energy"]])
    errs = {name: rel([got[i]], [ref[i]]) for i, name in enumerate(["total", "phys", "ic", "sym", "energy"])}
    errs["grad"] = rel(t2n(r["grad"]), grad)
    report(f"total loss via packed kernels: {case}", **errs)
    assert all(v < TOL for v in errs.values()), errs
