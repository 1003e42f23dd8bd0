"""The hybrid model's float64 reference on the CPU: the oracle's angle/Jacobian VJP inside torch
autograd passes gradcheck, and the hybrid model's classical parameter count matches the paper's
Table of parameter counts up to the learned time period of its periodic input mapping."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from tests.hybrid_reference import OracleAnglesFn, oracle_circuit_fn


def test_oracle_angles_function_passes_gradcheck():
    enc = W.Encoding(kind=W.ENC_ANGLES, gate=W.ENC_RX)
    circ = W.basic_entangling(3, 2, "rot", enc=enc)
    g = torch.Generator().manual_seed(0)
    params = (torch.rand(circ.n_params, generator=g, dtype=torch.float64) * 2 * math.pi).requires_grad_()
    theta = (torch.rand(2, 3, generator=g, dtype=torch.float64) * 3).requires_grad_()
    jac = torch.randn(2, 3, 3, generator=g, dtype=torch.float64).requires_grad_()
    assert torch.autograd.gradcheck(lambda p, t, j: OracleAnglesFn.apply(p, t, j, circ), (params, theta, jac),
                                    eps=1e-6, atol=1e-7)


def test_hybrid_model_parameter_counts():
    from paper_2506_23246_amd.hybrid import HybridQPINN
    import json
    import os
    circ = W.paper_context_circuit("basic")
    model = HybridQPINN(circ, circuit_fn=oracle_circuit_fn(circ), dtype=torch.float64)
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_param_counts.json")) as fh:
        table = json.load(fh)
    assert table["n_qubits"] == circ.n and table["quantum_params"]["basic"] == circ.n_params
    assert model.classical_parameter_count() + 1 == 66848        # + the learned time period
    assert model.quantum.params.numel() == circ.n_params == 84


def test_hybrid_reference_forward_backward_runs():
    from paper_2506_23246_amd.hybrid import HybridQPINN, maxwell_residual_loss
    circ = W.paper_context_circuit("basic")
    model = HybridQPINN(circ, circuit_fn=oracle_circuit_fn(circ), dtype=torch.float64, seed=1)
    pts = torch.tensor(np.random.default_rng(0).uniform(-1, 1, (3, 3)))
    fields, dfields = model(pts)
    loss = maxwell_residual_loss(dfields, pts)
    loss.backward()
    assert fields.shape == (3, 3) and dfields.shape == (3, 3, 3)
    # every parameter but the head's bias (the residuals see only the fields' derivatives)
    for name, p in model.named_parameters():
        if name != "head.bias":
            assert p.grad is not None and torch.isfinite(p.grad).all() and p.grad.abs().max() > 0, name


def test_hybrid_total_loss_terms_are_the_oracle_formulas():
    """The torch total loss of the hybrid model equals the oracle's total-loss function applied to
    the same model's fields and derivatives at the four point sets (float64, CPU)."""
    from oracle import qpinn_oracle as O
    from paper_2506_23246_amd.hybrid import HybridQPINN
    from paper_2506_23246_amd.train import hybrid_total_loss
    circ = W.paper_context_circuit("basic")
    model = HybridQPINN(circ, circuit_fn=oracle_circuit_fn(circ), dtype=torch.float64, seed=3)
    rng = np.random.default_rng(5)
    pts = torch.tensor(rng.uniform(-1, 1, (4, 3)))
    xy = torch.tensor(rng.uniform(-1, 1, (3, 2)))
    for kind in (W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT):
        desc = W.TotalLossDesc(phys=W.MaxwellDesc(kind, 4.0, 0.0))
        t = hybrid_total_loss(model, pts, xy, desc)
        f, g = (a.detach().numpy() for a in model(pts))
        f_mx = model.fields(torch.tensor(O.mirror_points(pts.numpy(), 1))).detach().numpy()
        f_my = model.fields(torch.tensor(O.mirror_points(pts.numpy(), 2))).detach().numpy()
        f_ic = model.fields(torch.tensor(O.ic_points(xy.numpy()))).detach().numpy()
        ref = O.total_loss(f, g, f_mx, f_my, f_ic, pts.numpy(), xy.numpy(), desc)
        for k in ("total", "phys", "ic", "sym", "energy"):
            assert float(t[k].detach()) == pytest.approx(ref[k], rel=1e-10, abs=1e-14), (kind, k)
