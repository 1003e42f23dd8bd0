"""The CPU oracle as a torch.autograd.Function over the angle-given encoding (test
infrastructure): forward = oracle outputs and input tangents, backward = the oracle's
stored-state reverse mode with respect to the parameters, the angles and their Jacobian.  It
stands in for the circuit engine when the hybrid model is evaluated as a float64 reference."""
import numpy as np
import torch

from oracle import qpinn_oracle as O


class OracleAnglesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, theta, jac, circ):
        prm = params.detach().cpu().numpy().astype(np.float64)
        th = theta.detach().cpu().numpy().astype(np.float64)
        J = jac.detach().cpu().numpy().astype(np.float64)
        f, g = O.simulate(circ, prm, None, th, J)
        ctx.save_for_backward(params, theta, jac)
        ctx.circ = circ
        return torch.tensor(f, dtype=theta.dtype), torch.tensor(g, dtype=theta.dtype)

    @staticmethod
    def backward(ctx, d_out, d_tan):
        params, theta, jac = ctx.saved_tensors
        m = len(ctx.circ.out_qubits)
        P = theta.shape[0]
        sf = np.zeros((P, m)) if d_out is None else d_out.detach().cpu().numpy().astype(np.float64)
        sg = np.zeros((P, m, 3)) if d_tan is None else d_tan.detach().cpu().numpy().astype(np.float64)
        g, d_th, d_J = O.grad_reverse(ctx.circ, params.detach().cpu().numpy().astype(np.float64), None, sf, sg,
                                      theta.detach().cpu().numpy().astype(np.float64),
                                      jac.detach().cpu().numpy().astype(np.float64), inputs=True)
        return (torch.tensor(g, dtype=params.dtype), torch.tensor(d_th, dtype=theta.dtype),
                torch.tensor(d_J, dtype=jac.dtype), None)


def oracle_circuit_fn(circ):
    """circuit_fn for paper_2506_23246_amd.hybrid.QuantumLayer backed by the oracle."""
    return lambda params, theta, jac: OracleAnglesFn.apply(params, theta, jac, circ)
