"""Seeded synthetic inputs for the QPINN circuit hot path.

This module is shared by the tests, ``bench.py`` and ``__graft_entry__.smoke()``.  It holds
circuit *descriptions* (ordered gate lists with parameter slots), the encoding and loss
descriptors, and seeded random draws of points, parameters and random-Fourier-feature
matrices.  It contains none of the method's arithmetic: no gate matrices, no simulation,
no readout, no loss.  Both the CPU oracle (``oracle/``) and the HIP path read the same
objects built here.

Conventions (readings of the paper, stated once):
  * qubit 0 is the most significant bit of a basis-state index (leftmost Kronecker factor);
  * a rotation gate R_P(theta) = exp(-i theta P / 2) with P in {X, Y, Z};
  * Rot(phi, theta, omega) = RZ(omega) RY(theta) RZ(phi) (section "QPINN architecture and
    ansatz designs", eq. rot_gate): RZ(phi) acts first, so it is emitted first;
  * a basic-entangling layer is one rotation block per qubit followed by the cyclic chain
    CNOT(q, (q+1) mod n), q = 0..n-1, applied in that order; the strongly-entangling layer
    widens the control-target gap by one per layer (same section), read here as a stride
    r_l = 1 + (l mod 3) for the CZ-ring workload;
  * collocation points are rows (t, x, y); column 0 is t.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# ---- gate kinds (shared numeric codes; the C header uses the same values) -------------
RX, RY, RZ, CNOT, CZ, CRZ = 0, 1, 2, 3, 4, 5
GATE_NAMES = {RX: "RX", RY: "RY", RZ: "RZ", CNOT: "CNOT", CZ: "CZ", CRZ: "CRZ"}
ROTATIONS = (RX, RY, RZ)

# ---- encoding descriptors ----------------------------------------------------------------
ENC_CYCLE, ENC_ANGLES, ENC_RFF = 0, 1, 2
ENC_RY, ENC_RX = 0, 1
SCALE_NONE, SCALE_PI, SCALE_BIAS, SCALE_ASIN, SCALE_ACOS = 0, 1, 2, 3, 4
SCALE_NAMES = {SCALE_NONE: "none", SCALE_PI: "pi", SCALE_BIAS: "bias",
               SCALE_ASIN: "asin", SCALE_ACOS: "acos"}

# ---- Maxwell loss descriptors --------------------------------------------------------------
LOSS_VACUUM, LOSS_DIEL_SPLIT, LOSS_DIEL_INTUITIVE = 0, 1, 2


@dataclass
class Encoding:
    """How a point (t, x, y) becomes one angle per qubit.

    kind=ENC_CYCLE : theta_q = scale(p[coord_of_qubit[q]]), coordinates cycled over qubits.
    kind=ENC_RFF   : phi = [cos(B p); sin(B p)], theta = W phi (B: [F,3], W: [n,2F]).
    kind=ENC_ANGLES: theta and its Jacobian d theta / d(t,x,y) are given per point.
    gate           : the embedding rotation applied to |0> (RY or RX).
    """
    kind: int = ENC_CYCLE
    gate: int = ENC_RY
    scale: int = SCALE_PI
    coord_of_qubit: list | None = None
    rff_B: np.ndarray | None = None
    rff_W: np.ndarray | None = None

    def coords(self, n: int) -> list:
        if self.coord_of_qubit is not None:
            return list(self.coord_of_qubit)
        return [q % 3 for q in range(n)]


@dataclass
class Circuit:
    n: int
    gates: list            # [(kind, q0, q1, param_index)], time order; q1 = -1 for 1-qubit gates
    n_params: int
    enc: Encoding = field(default_factory=Encoding)
    out_qubits: list = field(default_factory=lambda: [0, 1, 2])
    name: str = ""


@dataclass
class MaxwellDesc:
    """TE_z Maxwell residual loss (section "PINN architecture ...", residual equations)."""
    kind: int = LOSS_VACUUM
    eps_r: float = 4.0
    x_interface: float = 0.0


@dataclass
class TotalLossDesc:
    """The paper's total loss (eq. 2D_lossTot): L_phys + w_ic L_IC + w_sym L_sym + w_energy L_energy.

    phys   : the residual loss (vacuum or dielectric) of the collocation points;
    ic_a   : initial E_z pulse exp(-ic_a (x^2 + y^2)) at t = 0, H = 0 (eqs. pulse_IC_*, IC_loss);
    L_sym  : mirrored-point parity penalty (eq. 2D_symLoss); the x-mirror terms are left out for
             the dielectric losses (the dielectric breaks that symmetry);
    L_energy: mean square of the local Poynting residual (eq. energy_loss)."""
    phys: MaxwellDesc = field(default_factory=MaxwellDesc)
    w_ic: float = 10.0
    w_sym: float = 10.0
    w_energy: float = 10.0
    ic_a: float = 25.0


@dataclass
class Workload:
    name: str
    circuit: Circuit
    params: np.ndarray      # [K] float32 (or float64 for the FP64 plain config)
    points: np.ndarray      # [P,3] float32 (or float64)
    loss: MaxwellDesc | None
    angles: np.ndarray | None = None      # ENC_ANGLES only: [P,n]
    jac: np.ndarray | None = None         # ENC_ANGLES only: [P,n,3]
    meta: dict = field(default_factory=dict)


# ---- ansatz builders (gate lists only) ------------------------------------------------------

def _rot_block(gates, q, p0, kind):
    """Append one single-qubit rotation block on qubit q, parameters p0, p0+1, p0+2."""
    if kind == "xyz":       # RX, RY, RZ in time order
        gates += [(RX, q, -1, p0), (RY, q, -1, p0 + 1), (RZ, q, -1, p0 + 2)]
        return 3
    if kind == "rot":       # Rot(phi, theta, omega) = RZ(omega) RY(theta) RZ(phi)
        gates += [(RZ, q, -1, p0), (RY, q, -1, p0 + 1), (RZ, q, -1, p0 + 2)]
        return 3
    if kind == "x":
        gates.append((RX, q, -1, p0))
        return 1
    if kind == "xz":
        gates += [(RX, q, -1, p0), (RZ, q, -1, p0 + 1)]
        return 2
    raise ValueError(kind)


def ring(n: int, kind: int, stride: int = 1) -> list:
    """Cyclic entangler ring: gate(q, (q+stride) mod n) for q = 0..n-1, skipping q == target."""
    out = []
    for q in range(n):
        t = (q + stride) % n
        if t != q:
            out.append((kind, q, t, -1))
    return out


def layered(n: int, L: int, rot: str = "xyz", rings=None, name: str = "",
            enc: Encoding | None = None, out_qubits=None) -> Circuit:
    """L layers of [rotation block on every qubit, then rings[l] (a list of entangler gates)]."""
    gates, p = [], 0
    for l in range(L):
        for q in range(n):
            p += _rot_block(gates, q, p, rot)
        if rings is not None:
            gates += rings(l)
    return Circuit(n=n, gates=gates, n_params=p, enc=enc or Encoding(),
                   out_qubits=list(out_qubits) if out_qubits is not None else [0, 1, 2],
                   name=name)


def basic_entangling(n, L, rot="rot", **kw):
    return layered(n, L, rot, lambda l: ring(n, CNOT, 1), name=f"basic_{n}q{L}l", **kw)


def strongly_entangling(n, L, rot="rot", ent=CNOT, **kw):
    return layered(n, L, rot, lambda l: ring(n, ent, 1 + (l % 3)),
                   name=f"strong_{n}q{L}l", **kw)


def no_entanglement(n, L, rot="rot", **kw):
    return layered(n, L, rot, None, name=f"noent_{n}q{L}l", **kw)


def cross_mesh(n, L, rot="x", ent=CRZ, **kw):
    """Cross-Mesh family: a rotation block per qubit, then ent(i, j) for every ordered pair i != j
    (eq. crz_cross_mesh).  CRZ pairs carry one parameter each; CNOT pairs none."""
    gates, p = [], 0
    for l in range(L):
        for q in range(n):
            p += _rot_block(gates, q, p, rot)
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                if ent == CRZ:
                    gates.append((CRZ, i, j, p))
                    p += 1
                else:
                    gates.append((ent, i, j, -1))
    out = kw.pop("out_qubits", None)
    return Circuit(n=n, gates=gates, n_params=p, enc=kw.pop("enc", None) or Encoding(),
                   out_qubits=list(out) if out is not None else [0, 1, 2],
                   name=f"crossmesh_{rot}_{n}q{L}l")


# ---- seeded draws -----------------------------------------------------------------------------

def _rngs(k: int, count: int):
    ss = np.random.SeedSequence(1000 + k)
    return [np.random.default_rng(s) for s in ss.spawn(count)]


def uniform_points(rng, P: int, dtype=np.float32) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=(P, 3)).astype(dtype)


def ic_plane_points(rng, N: int, dtype=np.float32) -> np.ndarray:
    """(x, y) of initial-condition points, uniform in [-1, 1]^2 (the paper uses a 64 x 64 plane)."""
    return rng.uniform(-1.0, 1.0, size=(N, 2)).astype(dtype)


def uniform_params(rng, K: int, dtype=np.float32) -> np.ndarray:
    return rng.uniform(0.0, 2.0 * math.pi, size=K).astype(dtype)


CONFIG_NAMES = {
    0: "c1_plain_4q2l_fp64_1024",
    1: "c2_6q5l_cnot_vacuum_16384",
    2: "c3_8q10l_rff_cz_diel_65536",
    3: "c4_uneven_batch_32",
    4: "c5_12q8l_cnot_vacuum_262144",
}
FULL_P = {0: 1024, 1: 16384, 2: 65536, 4: 262144}


def config(k: int, P: int | None = None) -> Workload | list:
    """Workload k (0..4) with its seeded inputs; P truncates to the first P points of the full draw.

    k=3 returns a list of 32 Workloads (the uneven batch)."""
    if k == 3:
        return batch_config(P_cap=P)
    r_pts, r_par, r_B, r_W, _ = _rngs(k, 5)
    Pfull = FULL_P[k]
    if k == 0:
        circ = layered(4, 2, "xyz", lambda l: ring(4, CNOT, 1), name=CONFIG_NAMES[0],
                       out_qubits=[0, 1, 2, 3])
        pts = uniform_points(r_pts, Pfull, np.float64)
        prm = uniform_params(r_par, circ.n_params, np.float64)
        loss = None
    elif k == 1:
        circ = layered(6, 5, "xyz", lambda l: ring(6, CNOT, 1), name=CONFIG_NAMES[1])
        pts = uniform_points(r_pts, Pfull)
        prm = uniform_params(r_par, circ.n_params)
        loss = MaxwellDesc(LOSS_VACUUM)
    elif k == 2:
        F = 64
        B = r_B.standard_normal((F, 3)).astype(np.float32)
        W = (r_W.standard_normal((8, 2 * F)) / math.sqrt(2 * F)).astype(np.float32)
        enc = Encoding(kind=ENC_RFF, gate=ENC_RY, scale=SCALE_NONE, rff_B=B, rff_W=W)
        circ = layered(8, 10, "rot", lambda l: ring(8, CZ, 1 + (l % 3)),
                       name=CONFIG_NAMES[2], enc=enc)
        pts = uniform_points(r_pts, Pfull)
        prm = uniform_params(r_par, circ.n_params)
        loss = MaxwellDesc(LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=0.0)
    elif k == 4:
        circ = layered(12, 8, "xyz", lambda l: ring(12, CNOT, 1), name=CONFIG_NAMES[4])
        pts = uniform_points(r_pts, Pfull)
        prm = uniform_params(r_par, circ.n_params)
        loss = MaxwellDesc(LOSS_VACUUM)
    else:
        raise ValueError(k)
    if P is not None:
        pts = pts[:P].copy()
    return Workload(CONFIG_NAMES[k], circ, prm, pts, loss)


MULTITILE_P = 2 * 65536 + 4096 + 37


def multitile_config(P: int = MULTITILE_P) -> Workload:
    """A 4-qubit, 2-layer RX/RY/RZ + CNOT-ring circuit (the plain FP64 workload's circuit) in
    float32 with the vacuum Maxwell loss, at a point count that gives every persistent workgroup
    of the default launch two or more point tiles and leaves a ragged last tile."""
    r_pts, r_par = _rngs(10, 2)
    circ = layered(4, 2, "xyz", lambda l: ring(4, CNOT, 1), name="c1_circuit_f32_multitile",
                   out_qubits=[0, 1, 2, 3])
    return Workload(circ.name, circ, uniform_params(r_par, circ.n_params),
                    uniform_points(r_pts, P), MaxwellDesc(LOSS_VACUUM))


def batch_config(P_cap: int | None = None, count: int = 32) -> list:
    """The uneven batch: per circuit n ~ U{4..10}, L ~ U{2..12}, P log-uniform in [1024, 65536],
    one ring type per layer ~ U{CNOT, CZ} (stride 1), RX/RY/RZ blocks, cycled RY encoding,
    vacuum Maxwell loss.  P_cap (if given) truncates every circuit's points."""
    r_draw, r_pts, r_par = _rngs(3, 3)
    out = []
    for c in range(count):
        n = int(r_draw.integers(4, 11))
        L = int(r_draw.integers(2, 13))
        P = int(round(math.exp(r_draw.uniform(math.log(1024), math.log(65536)))))
        kinds = [CNOT if r_draw.integers(0, 2) == 0 else CZ for _ in range(L)]
        circ = layered(n, L, "xyz", lambda l, kinds=kinds, n=n: ring(n, kinds[l], 1),
                       name=f"batch{c:02d}_{n}q{L}l")
        pts = uniform_points(r_pts, P)
        prm = uniform_params(r_par, circ.n_params)
        if P_cap is not None:
            pts = pts[:P_cap].copy()
        out.append(Workload(circ.name, circ, prm, pts, MaxwellDesc(LOSS_VACUUM),
                            meta={"ring_kinds": kinds, "P_full": P}))
    return out


def paper_context_circuit(ansatz: str = "basic", n: int = 7, L: int = 4) -> Circuit:
    """The paper's PQC shape: 7 qubits, 4 layers, RX angle embedding, <Z> of every qubit read out
    (section "QPINN architecture": each qubit acts as a neuron of the layer)."""
    enc = Encoding(kind=ENC_ANGLES, gate=ENC_RX, scale=SCALE_ACOS)
    circ = _paper_ansatz(ansatz, n, L, enc)
    circ.out_qubits = list(range(n))
    return circ


def _paper_ansatz(ansatz, n, L, enc):
    if ansatz == "basic":
        return basic_entangling(n, L, "rot", enc=enc)
    if ansatz == "strong":
        return strongly_entangling(n, L, "rot", enc=enc)
    if ansatz == "noent":
        return no_entanglement(n, L, "rot", enc=enc)
    if ansatz == "cross_mesh":
        return cross_mesh(n, L, "x", CRZ, enc=enc)
    if ansatz == "cross_mesh_2rot":
        return cross_mesh(n, L, "xz", CRZ, enc=enc)
    if ansatz == "cross_mesh_cnot":
        return cross_mesh(n, L, "rot", CNOT, enc=enc)
    raise ValueError(ansatz)
