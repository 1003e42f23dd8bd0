"""torch.autograd.Function over the circuit engine.

forward  -> qp_simulate : outputs <Z_i> [P,m] and input tangents d<Z_i>/d(t,x,y) [P,m,3]
backward -> qp_vjp      : gradients from the incoming gradients of both outputs, by the adjoint
                          sweep that uncomputes the forward with inverse gates (no stored states).

Two input forms:
* points [P,3] with a point encoding (cycled coordinates, random Fourier features): the points
  are not differentiated (their derivatives are what the tangents already provide); gradients
  flow to the parameters only;
* angles [P,n] and their Jacobian [P,n,3] with respect to (t, x, y) (the angle-given encoding,
  a classical layer in front of the circuit as in the paper's hybrid model, section "QPINN
  architecture and ansatz designs"): gradients flow to the parameters, the angles and the
  Jacobian, and from there back into the layer that produced them.
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


class QCircuitAnglesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, angles, jac, circuit: Circuit):
        out, tan = circuit.simulate(params, None, angles=angles, jac=jac)
        ctx.circuit = circuit
        ctx.save_for_backward(params, angles, jac)
        return out, tan

    @staticmethod
    def backward(ctx, d_out, d_tan):
        params, angles, jac = ctx.saved_tensors
        need = ctx.needs_input_grad
        if not any(need[:3]):
            return None, None, None, None
        ig = bool(need[1] or need[2])
        r = ctx.circuit.vjp(params, None,
                            None if d_out is None else d_out.contiguous(),
                            None if d_tan is None else d_tan.contiguous(),
                            angles=angles, jac=jac, input_grads=ig)
        g, ga, gj = r if ig else (r, None, None)
        return (g if need[0] else None, ga if need[1] else None, gj if need[2] else None, None)


def qcircuit(params, points, circuit: Circuit):
    """(out, tan) with gradients flowing to params."""
    return QCircuitFn.apply(params, points, circuit)


def qcircuit_angles(params, angles, jac, circuit: Circuit):
    """(out, tan) of the angle-given encoding, with gradients flowing to params, angles and jac."""
    return QCircuitAnglesFn.apply(params, angles, jac, circuit)
