"""The paper's hybrid QPINN as torch modules around the circuit engine (section "QPINN
architecture and ansatz designs"): a classical network maps (t, x, y) to one activation per
qubit, the activations are scaled to angles (eq. scale) and angle-embedded, the parametrised
circuit is read out as <Z_i>, and a linear head maps the n readouts to (E_z, H_x, H_y).

The Maxwell residuals need the fields' derivatives in (t, x, y).  Here they are formed without
differentiating through the circuit: the angle Jacobian J = d angles / d(t, x, y) comes from the
classical network (torch autograd, kept in the graph), the circuit engine carries it forward as
tangent statevectors and returns d<Z_i>/d(t, x, y), and the linear head maps those like the
readouts.  In the backward pass the engine's adjoint returns the gradients with respect to the
circuit parameters, the angles and the Jacobian (qp_vjp), and torch carries them on into the
classical network.

Classical part (section "PINN architecture and convergence enhancements"): random Fourier
features of the inputs (64 fixed Gaussian frequencies, cos and sin: 128 features), a first
hidden layer of 256 neurons, then hidden layers of 128, tanh activations; the layer before the
head is replaced by the circuit (7 qubits, 4 layers in the paper).  With one hidden layer of 128
after the 256 one this has 66847 trainable classical parameters; the paper's count of 66848 also
includes the learned time period of its periodic input mapping, which is not part of this build.
"""
from __future__ import annotations

import math

import torch
from torch import nn

from .api import Circuit, Context
from .autograd import qcircuit_angles

SCALE_NONE, SCALE_PI, SCALE_BIAS, SCALE_ASIN, SCALE_ACOS = 0, 1, 2, 3, 4


def scale_angles(kind: int, a: torch.Tensor) -> torch.Tensor:
    """Input scalings of eq. scale applied to activations a in (-1, 1): a, pi a, (a + 1) pi/2,
    asin(a) + pi/2, acos(a)."""
    if kind == SCALE_NONE:
        return a
    if kind == SCALE_PI:
        return math.pi * a
    if kind == SCALE_BIAS:
        return (a + 1.0) * (math.pi / 2.0)
    if kind == SCALE_ASIN:
        return torch.asin(a) + math.pi / 2.0
    if kind == SCALE_ACOS:
        return torch.acos(a)
    raise ValueError(kind)


def input_jacobian(theta: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """J[p, q, c] = d theta[p, q] / d x[p, c] for a map applied point by point, kept in the graph
    (create_graph) so that a loss on J differentiates into the map's weights."""
    cols = []
    for q in range(theta.shape[1]):
        (g,) = torch.autograd.grad(theta[:, q].sum(), x, create_graph=True)
        cols.append(g)
    return torch.stack(cols, dim=1)


class QuantumLayer(nn.Module):
    """Angle embedding + ansatz + Pauli-Z readout on the circuit engine.

    forward(theta [P,n], jac [P,n,3]) -> (out [P,m], tan [P,m,3]); gradients flow to the circuit
    parameters, theta and jac.  `circuit` is a circuit description with the angle-given encoding
    (workloads.Circuit or any object with n, gates, n_params, enc, out_qubits)."""

    def __init__(self, circuit, ctx: Context | None = None, params: torch.Tensor | None = None,
                 circuit_fn=None, dtype=torch.float32):
        super().__init__()
        self.desc = circuit
        if params is None:
            params = torch.rand(circuit.n_params) * (2 * math.pi)
        self.params = nn.Parameter(torch.as_tensor(params).to(dtype).clone())
        self._fn = circuit_fn
        self._circ = None
        if circuit_fn is None:
            self._circ = Circuit(ctx if ctx is not None else Context(0), circuit)

    def forward(self, theta, jac):
        if self._fn is not None:      # another implementation of the same layer (a reference)
            return self._fn(self.params, theta, jac)
        return qcircuit_angles(self.params, theta.float().contiguous(), jac.float().contiguous(), self._circ)


class HybridQPINN(nn.Module):
    """RFF -> Linear(128, 256) -> tanh -> Linear(256, 128) -> tanh -> Linear(128, n) -> tanh ->
    scale -> quantum layer (n readouts) -> Linear(m, 3) = (E_z, H_x, H_y)."""

    def __init__(self, circuit, scale: int = SCALE_ACOS, n_freq: int = 64, hidden=(256, 128),
                 ctx: Context | None = None, seed: int = 0, circuit_fn=None, dtype=torch.float32):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        self.register_buffer("B", torch.randn(n_freq, 3, generator=g, dtype=dtype))
        dims = [2 * n_freq, *hidden, circuit.n]
        self.layers = nn.ModuleList(nn.Linear(a, b, dtype=dtype) for a, b in zip(dims[:-1], dims[1:]))
        self.scale = scale
        self.quantum = QuantumLayer(circuit, ctx, circuit_fn=circuit_fn,
                                    dtype=dtype if circuit_fn is not None else torch.float32)
        self.head = nn.Linear(len(circuit.out_qubits), 3, dtype=dtype)

    def angles(self, x):
        proj = x @ self.B.T
        h = torch.cat([torch.cos(proj), torch.sin(proj)], dim=1)
        for i, lin in enumerate(self.layers):
            h = torch.tanh(lin(h))
        return scale_angles(self.scale, h)

    def forward(self, points):
        """Fields [P,3] and their derivatives d field_i / d(t, x, y) [P,3,3]."""
        x = points.detach().clone().requires_grad_(True)
        theta = self.angles(x)
        jac = input_jacobian(theta, x)
        out, tan = self.quantum(theta, jac)
        out, tan = out.to(self.head.weight.dtype), tan.to(self.head.weight.dtype)
        fields = self.head(out)
        dfields = torch.einsum("fi,pic->pfc", self.head.weight, tan)
        return fields, dfields

    def fields(self, points):
        """Fields [P,3] alone (no input derivatives: the circuit gets a zero Jacobian)."""
        theta = self.angles(points)
        jac = torch.zeros(theta.shape + (3,), dtype=theta.dtype, device=theta.device)
        out, _ = self.quantum(theta, jac)
        return self.head(out.to(self.head.weight.dtype))

    def classical_parameter_count(self) -> int:
        return sum(p.numel() for n, p in self.named_parameters() if not n.startswith("quantum."))


def maxwell_residual_loss(dfields: torch.Tensor, points: torch.Tensor, kind: int = 0, eps_r: float = 4.0,
                          x_interface: float = 0.0) -> torch.Tensor:
    """TE_z Maxwell residuals from the field derivatives (eqs. residual_1_vac, residual_1_diel,
    residuals_2_and_3) and their MSE loss (eqs. phys_loss_vac, phys_loss_diel): kind 0 vacuum,
    1 split dielectric (separate means over x < x_interface and x >= x_interface)."""
    dE, dHx, dHy = dfields[:, 0], dfields[:, 1], dfields[:, 2]
    diel = points[:, 1] >= x_interface
    eps = torch.where(diel, torch.full_like(dE[:, 0], eps_r), torch.ones_like(dE[:, 0])) if kind else torch.ones_like(dE[:, 0])
    r1 = dE[:, 0] - (dHy[:, 1] - dHx[:, 2]) / eps
    r2 = dHx[:, 0] + dE[:, 2]
    r3 = dHy[:, 0] - dE[:, 1]
    if kind == 1:
        l1 = sum(torch.mean(r1[m] ** 2) for m in (~diel, diel) if bool(m.any()))
    else:
        l1 = torch.mean(r1 ** 2)
    return l1 + torch.mean(r2 ** 2) + torch.mean(r3 ** 2)
