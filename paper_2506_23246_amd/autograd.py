"""torch.autograd.Function over the circuit engine.

forward  -> qp_simulate : outputs <Z_i> [P,m] and input tangents d<Z_i>/d(t,x,y) [P,m,3]
backward -> qp_vjp      : d params from the incoming gradients of both outputs, by the adjoint
                          sweep that uncomputes the forward with inverse gates (no stored states).
The points are not differentiated (their derivatives are what the tangents already provide).
"""
from __future__ import annotations

import torch

from .api import Circuit


class QCircuitFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, points, circuit: Circuit):
        out, tan = circuit.simulate(params, points)
        ctx.circuit = circuit
        ctx.save_for_backward(params, points)
        return out, tan

    @staticmethod
    def backward(ctx, d_out, d_tan):
        params, points = ctx.saved_tensors
        g = None
        if ctx.needs_input_grad[0]:
            g = ctx.circuit.vjp(params, points,
                                None if d_out is None else d_out.contiguous(),
                                None if d_tan is None else d_tan.contiguous())
        return g, None, None


def qcircuit(params, points, circuit: Circuit):
    """(out, tan) with gradients flowing to params."""
    return QCircuitFn.apply(params, points, circuit)
