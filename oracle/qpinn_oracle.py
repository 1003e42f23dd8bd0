"""Plain CPU complex128 oracle for the QPINN circuit hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code with the HIP
path (no kernels, tables, helpers or constants); the two meet only through the seeded inputs
of ``workloads.py``.

It follows the paper's definitions one step at a time, slowly and visibly:

* angle embedding of each collocation point, with the five input scalings of eq. ``scale``
  (section "QPINN architecture and ansatz designs") or random Fourier features
  (section "PINN architecture and convergence enhancements", RFF item);
* every gate is turned into its full 2^n x 2^n operator by an explicit Kronecker product
  (dense ``np.kron`` for n <= 8, ``scipy.sparse.kron`` beyond) and applied, unfused and in
  time order, to the state and to its three input-tangent states;
* the Pauli-Z readout of each qubit (same section: each qubit acts as a neuron);
* the TE_z Maxwell residuals and MSE losses (eqs. residual_1_vac, residual_1_diel,
  residuals_2_and_3, phys_loss_vac, phys_loss_diel, mse, residual_1_intuitive);
* parameter gradients of the loss by three independent routes: stored-state reverse mode,
  the parameter-shift rule (section "QPINN architecture": the hardware-compatible method)
  applied to the readouts, and central finite differences of the loss.

Readings of the paper that it fixes (the paper does not define them):
  R_P(theta) = exp(-i theta P / 2); qubit 0 is the leftmost Kronecker factor; the fields are
  (E_z, H_x, H_y) = (<Z_{o0}>, <Z_{o1}>, <Z_{o2}>) for the first three output qubits.

Precision: float64 / complex128 throughout; inputs given as float32 are upcast exactly.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# gate / encoding / loss codes are data shared with the inputs module (numbers only)
RX, RY, RZ, CNOT, CZ, CRZ = 0, 1, 2, 3, 4, 5
ENC_CYCLE, ENC_ANGLES, ENC_RFF = 0, 1, 2
ENC_RY, ENC_RX = 0, 1
SCALE_NONE, SCALE_PI, SCALE_BIAS, SCALE_ASIN, SCALE_ACOS = 0, 1, 2, 3, 4
LOSS_VACUUM, LOSS_DIEL_SPLIT, LOSS_DIEL_INTUITIVE = 0, 1, 2

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
PAULI = {RX: PX, RY: PY, RZ: PZ}

DENSE_MAX_N = 8


# ---------------------------------------------------------------- gates -----------------------

def rotation(kind: int, theta: float) -> np.ndarray:
    """R_P(theta) = exp(-i theta P/2) = cos(theta/2) I - i sin(theta/2) P."""
    return math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * PAULI[kind]


def rotation_derivative(kind: int, theta: float) -> np.ndarray:
    """d/dtheta R_P(theta) = -(i/2) P R_P(theta)."""
    return -0.5j * PAULI[kind] @ rotation(kind, theta)


def _kron_list(factors, sparse: bool):
    out = factors[0]
    if sparse:
        out = sp.csr_matrix(out)
        for f in factors[1:]:
            out = sp.kron(out, sp.csr_matrix(f), format="csr")
        return out
    for f in factors[1:]:
        out = np.kron(out, f)
    return out


def full_operator(n: int, kind: int, q0: int, q1: int, theta: float | None,
                  derivative: bool = False):
    """The gate as a full 2^n x 2^n operator, built by an explicit Kronecker product.

    Single-qubit: I (x) ... (x) U (x) ... (x) I with U in slot q0.
    CNOT(c,t) = P0^(c) (x) I + P1^(c) (x) X^(t);  CZ(a,b) = P0^(a) (x) I + P1^(a) (x) Z^(b);
    CRZ(c,t)  = P0^(c) (x) I + P1^(c) (x) RZ(theta)^(t).
    With derivative=True the operator is d(gate)/d(theta) (parametrised gates only).
    """
    sparse = n > DENSE_MAX_N
    if kind in (RX, RY, RZ):
        U = rotation_derivative(kind, theta) if derivative else rotation(kind, theta)
        return _kron_list([U if q == q0 else I2 for q in range(n)], sparse)
    if kind in (CNOT, CZ, CRZ):
        if kind == CNOT:
            T = PX
        elif kind == CZ:
            T = PZ
        else:
            T = rotation_derivative(RZ, theta) if derivative else rotation(RZ, theta)
        zero_branch = [P0 if q == q0 else I2 for q in range(n)]
        one_branch = [P1 if q == q0 else (T if q == q1 else I2) for q in range(n)]
        if derivative:      # only the controlled branch depends on theta
            return _kron_list(one_branch, sparse)
        return _kron_list(zero_branch, sparse) + _kron_list(one_branch, sparse)
    raise ValueError(f"unknown gate kind {kind}")


def z_diagonal(n: int, i: int) -> np.ndarray:
    """Diagonal of Z_i^full = I (x) .. (x) Z (slot i) (x) .. (x) I, by explicit Kronecker product."""
    d = np.ones(1)
    for q in range(n):
        d = np.kron(d, np.array([1.0, -1.0]) if q == i else np.ones(2))
    return d


# ------------------------------------------------------------- encoding -----------------------

def scale_value(kind: int, a):
    """Input scalings, eq. scale: none, pi, bias, asin, acos."""
    if kind == SCALE_NONE:
        return a
    if kind == SCALE_PI:
        return math.pi * a
    if kind == SCALE_BIAS:
        return (a + 1.0) * math.pi / 2.0
    if kind == SCALE_ASIN:
        return np.arcsin(a) + math.pi / 2.0
    if kind == SCALE_ACOS:
        return np.arccos(a)
    raise ValueError(kind)


def scale_derivative(kind: int, a):
    if kind == SCALE_NONE:
        return np.ones_like(a)
    if kind == SCALE_PI:
        return np.full_like(a, math.pi)
    if kind == SCALE_BIAS:
        return np.full_like(a, math.pi / 2.0)
    if kind == SCALE_ASIN:
        return 1.0 / np.sqrt(1.0 - a * a)
    if kind == SCALE_ACOS:
        return -1.0 / np.sqrt(1.0 - a * a)
    raise ValueError(kind)


def encoding_angles(circ, points, angles=None, jac=None):
    """theta [P,n] and J = d theta / d(t,x,y) [P,n,3] for every point (float64)."""
    enc = circ.enc
    if enc.kind == ENC_ANGLES:      # angles given per point; the points themselves are not read
        return np.asarray(angles, np.float64).copy(), np.asarray(jac, np.float64).copy()
    pts = np.asarray(points, dtype=np.float64)
    P, n = pts.shape[0], circ.n
    if enc.kind == ENC_CYCLE:
        coords = enc.coords(n)
        theta = np.empty((P, n))
        J = np.zeros((P, n, 3))
        for q in range(n):
            a = pts[:, coords[q]]
            theta[:, q] = scale_value(enc.scale, a)
            J[:, q, coords[q]] = scale_derivative(enc.scale, a)
        return theta, J
    if enc.kind == ENC_RFF:
        # phi = [cos(B p); sin(B p)] (fixed Gaussian B), theta = W phi
        B = np.asarray(enc.rff_B, np.float64)          # [F,3]
        W = np.asarray(enc.rff_W, np.float64)          # [n,2F]
        proj = pts @ B.T                               # [P,F]
        phi = np.concatenate([np.cos(proj), np.sin(proj)], axis=1)
        theta = phi @ W.T
        # d phi / d p: [P,2F,3]
        dphi = np.concatenate([-np.sin(proj)[:, :, None] * B[None],
                               np.cos(proj)[:, :, None] * B[None]], axis=1)
        J = np.einsum("qf,pfc->pqc", W, dphi)
        return theta, J
    raise ValueError(enc.kind)


def _embed_vectors(gate: int, theta):
    """Single-qubit embedded state G(theta)|0> and its theta-derivative, for an array of angles."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    if gate == ENC_RY:
        v = np.stack([c, s], -1).astype(np.complex128)
        dv = np.stack([-0.5 * s, 0.5 * c], -1).astype(np.complex128)
    else:   # RX: (cos, -i sin)
        v = np.stack([c + 0j, -1j * s], -1)
        dv = np.stack([-0.5 * s + 0j, -0.5j * c], -1)
    return v, dv


def _embed_second_derivative(gate: int, theta):
    """d^2/dtheta^2 of the embedded state: RY (cos, sin)(theta/2) -> -(1/4)(cos, sin);
    RX (cos, -i sin)(theta/2) -> -(1/4)(cos, -i sin)."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    if gate == ENC_RY:
        return np.stack([-0.25 * c, -0.25 * s], -1).astype(np.complex128)
    return np.stack([-0.25 * c + 0j, 0.25j * s], -1)


def initial_states(circ, theta, J):
    """psi0 = kron_q G(theta_q)|0> and the tangents dpsi0_c = sum_q J_qc kron(.., dG_q|0>, ..).

    Returns psi [2^n, P] and dpsi [3, 2^n, P] (one column per point)."""
    P, n = theta.shape
    v, dv = _embed_vectors(circ.enc.gate, theta)          # [P,n,2]
    psi = np.zeros((2 ** n, P), np.complex128)
    dpsi = np.zeros((3, 2 ** n, P), np.complex128)
    for p in range(P):
        factors = [v[p, q] for q in range(n)]
        psi[:, p] = _kron_list(factors, False)
        for q in range(n):
            if not np.any(J[p, q] != 0.0):
                continue
            term = _kron_list([dv[p, q] if qq == q else v[p, qq] for qq in range(n)], False)
            for c in range(3):
                if J[p, q, c] != 0.0:
                    dpsi[c, :, p] += J[p, q, c] * term
    return psi, dpsi


# ------------------------------------------------------------ simulation ----------------------

def _param_angle(params, g):
    kind, q0, q1, pi = g
    return float(params[pi]) if pi >= 0 else None


def operators(circ, params, derivative=False):
    """Full operators for every gate, in time order (cached per call)."""
    out = []
    for g in circ.gates:
        kind, q0, q1, pi = g
        th = _param_angle(params, g)
        if derivative and pi < 0:
            out.append(None)
        else:
            out.append(full_operator(circ.n, kind, q0, q1, th, derivative))
    return out


def readout(circ, psi, dpsi):
    """f_i = Re psi^H Z_i psi, g_ic = 2 Re psi^H Z_i dpsi_c for the output qubits."""
    outs = circ.out_qubits
    P = psi.shape[1]
    f = np.zeros((P, len(outs)))
    g = np.zeros((P, len(outs), 3))
    for k, i in enumerate(outs):
        z = z_diagonal(circ.n, i)[:, None]
        f[:, k] = np.real(np.sum(np.conj(psi) * z * psi, axis=0))
        for c in range(3):
            g[:, k, c] = 2.0 * np.real(np.sum(np.conj(psi) * z * dpsi[c], axis=0))
    return f, g


def simulate(circ, params, points, angles=None, jac=None, chunk=256):
    """Outputs f [P,m] and input tangents g [P,m,3] (float64)."""
    params = np.asarray(params, np.float64)
    theta, J = encoding_angles(circ, points, angles, jac)
    ops = operators(circ, params)
    P = theta.shape[0]
    f = np.zeros((P, len(circ.out_qubits)))
    g = np.zeros((P, len(circ.out_qubits), 3))
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        psi, dpsi = initial_states(circ, theta[s:e], J[s:e])
        for U in ops:
            psi = U @ psi
            for c in range(3):
                dpsi[c] = U @ dpsi[c]
        f[s:e], g[s:e] = readout(circ, psi, dpsi)
    return f, g


def final_states(circ, params, points, angles=None, jac=None):
    params = np.asarray(params, np.float64)
    theta, J = encoding_angles(circ, points, angles, jac)
    psi, dpsi = initial_states(circ, theta, J)
    for U in operators(circ, params):
        psi = U @ psi
        for c in range(3):
            dpsi[c] = U @ dpsi[c]
    return psi, dpsi


# ------------------------------------------------------------------ loss ----------------------

def maxwell_terms(g, points, desc):
    """Residuals and per-point weights of the TE_z Maxwell loss.

    With (E_z, H_x, H_y) the first three outputs and g[:, i, c] = d field_i / d coordinate c
    (c = 0:t, 1:x, 2:y):
      r1 = dE/dt - (1/eps)(dHy/dx - dHx/dy)   (eqs. residual_1_vac / residual_1_diel / intuitive)
      r2 = dHx/dt + dE/dy,  r3 = dHy/dt - dE/dx  (eq. residuals_2_and_3)
    Loss = sum_p w1_p r1_p^2 + (1/P) sum_p (r2_p^2 + r3_p^2), with
      vacuum:      eps = 1, w1 = 1/P                                   (eq. phys_loss_vac)
      split:       eps = 1, w1 = 1/N_vac for x < x_if;  eps = eps_r, w1 = 1/N_diel otherwise
                   (eq. phys_loss_diel with eq. mse; an empty region contributes nothing)
      intuitive:   eps(x) as above, w1 = 1/P                           (eq. phys_loss_intuitive)
    """
    pts = np.asarray(points, np.float64)
    P = pts.shape[0]
    diel = pts[:, 1] >= desc.x_interface
    if desc.kind == LOSS_VACUUM:
        eps = np.ones(P)
        w1 = np.full(P, 1.0 / P)
    else:
        eps = np.where(diel, desc.eps_r, 1.0)
        if desc.kind == LOSS_DIEL_SPLIT:
            n_d = int(diel.sum())
            n_v = P - n_d
            w1 = np.where(diel, 1.0 / max(n_d, 1), 1.0 / max(n_v, 1))
        else:
            w1 = np.full(P, 1.0 / P)
    w = np.full(P, 1.0 / P)
    dE, dHx, dHy = g[:, 0, :], g[:, 1, :], g[:, 2, :]
    r1 = dE[:, 0] - (dHy[:, 1] - dHx[:, 2]) / eps
    r2 = dHx[:, 0] + dE[:, 2]
    r3 = dHy[:, 0] - dE[:, 1]
    return r1, r2, r3, eps, w1, w


def maxwell_loss(g, points, desc):
    r1, r2, r3, eps, w1, w = maxwell_terms(g, points, desc)
    return float(np.sum(w1 * r1 ** 2) + np.sum(w * (r2 ** 2 + r3 ** 2)))


def maxwell_seeds(g, points, desc):
    """W[p, i, c] = d Loss / d g[p, i, c] (the loss is a quadratic form in g)."""
    r1, r2, r3, eps, w1, w = maxwell_terms(g, points, desc)
    W = np.zeros_like(g)
    a = 2.0 * w1 * r1
    W[:, 0, 0] += a
    W[:, 2, 1] += -a / eps
    W[:, 1, 2] += a / eps
    b = 2.0 * w * r2
    W[:, 1, 0] += b
    W[:, 0, 2] += b
    c = 2.0 * w * r3
    W[:, 2, 0] += c
    W[:, 0, 1] += -c
    return W


# ------------------------------------------------------- the paper's total loss ---------------
#
# L_tot = L_phys + w_ic L_IC + w_sym L_sym + w_energy L_energy (eq. 2D_lossTot, weights 1/10/10/10)
# over three point sets: the collocation points X (residuals, energy), their mirror images
# X_mx = (t, -x, y) and X_my = (t, x, -y) (symmetry), and the initial-condition plane X_0 = (0, x, y).

def mirror_points(points, axis: int):
    """(t, -x, y) for axis 1, (t, x, -y) for axis 2."""
    out = np.array(points, dtype=np.float64, copy=True)
    out[:, axis] = -out[:, axis]
    return out


def ic_points(ic_xy):
    """(t, x, y) = (0, x, y) for the initial-condition plane."""
    xy = np.asarray(ic_xy, np.float64)
    return np.concatenate([np.zeros((xy.shape[0], 1)), xy], axis=1)


def _eps(points, desc):
    pts = np.asarray(points, np.float64)
    if desc.kind == LOSS_VACUUM:
        return np.ones(pts.shape[0])
    return np.where(pts[:, 1] >= desc.x_interface, desc.eps_r, 1.0)


def energy_residual(f, g, points, desc):
    """Local Poynting residual (eqs. Poynting_thm, Poynting_value_u, Poynting_value_S, energy_loss)
    with u = (eps E^2 + Hx^2 + Hy^2)/2, S = (-E Hy, E Hx), J = 0:
      e = eps E dE/dt + Hx dHx/dt + Hy dHy/dt - (dE/dx Hy + E dHy/dx) + (dE/dy Hx + E dHx/dy)."""
    eps = _eps(points, desc)
    E, Hx, Hy = f[:, 0], f[:, 1], f[:, 2]
    Et, Ex, Ey = g[:, 0, 0], g[:, 0, 1], g[:, 0, 2]
    Hxt, Hxy = g[:, 1, 0], g[:, 1, 2]
    Hyt, Hyx = g[:, 2, 0], g[:, 2, 1]
    return (eps * E * Et + Hx * Hxt + Hy * Hyt) - (Ex * Hy + E * Hyx) + (Ey * Hx + E * Hxy)


def ic_target(ic_xy, a):
    xy = np.asarray(ic_xy, np.float64)
    return np.exp(-a * (xy[:, 0] ** 2 + xy[:, 1] ** 2))


def _sym_terms(f, f_mx, f_my, desc):
    """Per-point squared parity defects of eq. 2D_symLoss: E even in x and y, H_x even in x and odd
    in y, H_y odd in x and even in y; the x-mirror terms only for the vacuum loss."""
    terms = (f[:, 0] - f_my[:, 0]) ** 2 + (f[:, 1] + f_my[:, 1]) ** 2 + (f[:, 2] - f_my[:, 2]) ** 2
    if desc.phys.kind == LOSS_VACUUM:
        terms = terms + (f[:, 0] - f_mx[:, 0]) ** 2 + (f[:, 1] - f_mx[:, 1]) ** 2 + (f[:, 2] + f_mx[:, 2]) ** 2
    return terms


def total_loss(f, g, f_mx, f_my, f_ic, points, ic_xy, desc):
    """The four terms and their weighted sum (eq. 2D_lossTot).  L_IC = mean over the plane of
    (E - E_0)^2 + Hx^2 + Hy^2 (eq. IC_loss); L_sym = mean over X of the parity defects; L_energy =
    mean over X of the squared Poynting residual (the paper prints the residual; it is squared and
    averaged here like every other residual)."""
    P = f.shape[0]
    phys = maxwell_loss(g, points, desc.phys) if P else 0.0
    E0 = ic_target(ic_xy, desc.ic_a)
    ic = float(np.mean((f_ic[:, 0] - E0) ** 2 + f_ic[:, 1] ** 2 + f_ic[:, 2] ** 2)) if len(E0) else 0.0
    sym = float(np.mean(_sym_terms(f, f_mx, f_my, desc))) if P else 0.0
    energy = float(np.mean(energy_residual(f, g, points, desc.phys) ** 2)) if P else 0.0
    total = phys + desc.w_ic * ic + desc.w_sym * sym + desc.w_energy * energy
    return {"total": total, "phys": phys, "ic": ic, "sym": sym, "energy": energy}


def total_loss_seeds(f, g, f_mx, f_my, f_ic, points, ic_xy, desc):
    """d L_tot / d(f, g) on every set, differentiated by hand from total_loss:
    returns (Vf [P,m], Wg [P,m,3], V_mx [P,m], V_my [P,m], V_ic [P0,m]); only the first three
    outputs (E_z, H_x, H_y) carry seeds."""
    P, m = f.shape
    Vf = np.zeros((P, m))
    Wg = maxwell_seeds(g, points, desc.phys) if P else np.zeros((0, m, 3))
    V_mx = np.zeros((P, m))
    V_my = np.zeros((P, m))
    # energy: w_energy * mean(e^2)
    if P:
        eps = _eps(points, desc.phys)
        e = energy_residual(f, g, points, desc.phys)
        k = desc.w_energy * 2.0 * e / P
        E, Hx, Hy = f[:, 0], f[:, 1], f[:, 2]
        Et, Ex, Ey = g[:, 0, 0], g[:, 0, 1], g[:, 0, 2]
        Hxt, Hxy = g[:, 1, 0], g[:, 1, 2]
        Hyt, Hyx = g[:, 2, 0], g[:, 2, 1]
        Vf[:, 0] += k * (eps * Et - Hyx + Hxy)
        Vf[:, 1] += k * (Hxt + Ey)
        Vf[:, 2] += k * (Hyt - Ex)
        Wg[:, 0, 0] += k * eps * E
        Wg[:, 0, 1] += -k * Hy
        Wg[:, 0, 2] += k * Hx
        Wg[:, 1, 0] += k * Hx
        Wg[:, 1, 2] += k * E
        Wg[:, 2, 0] += k * Hy
        Wg[:, 2, 1] += -k * E
        # symmetry: w_sym * mean(defects); d (a - s b)^2 = 2 (a - s b) (da - s db)
        ks = desc.w_sym * 2.0 / P
        for i, s in enumerate((1.0, -1.0, 1.0)):          # y-mirror parities of E, Hx, Hy
            d = f[:, i] - s * f_my[:, i]
            Vf[:, i] += ks * d
            V_my[:, i] += -ks * s * d
        if desc.phys.kind == LOSS_VACUUM:
            for i, s in enumerate((1.0, 1.0, -1.0)):      # x-mirror parities
                d = f[:, i] - s * f_mx[:, i]
                Vf[:, i] += ks * d
                V_mx[:, i] += -ks * s * d
    P0 = f_ic.shape[0]
    V_ic = np.zeros((P0, m))
    if P0:
        ki = desc.w_ic * 2.0 / P0
        V_ic[:, 0] = ki * (f_ic[:, 0] - ic_target(ic_xy, desc.ic_a))
        V_ic[:, 1] = ki * f_ic[:, 1]
        V_ic[:, 2] = ki * f_ic[:, 2]
    return Vf, Wg, V_mx, V_my, V_ic


def total_eval(circ, params, points, ic_xy, desc):
    """Forward on the four sets, the total loss and its parameter gradient (reverse mode on each
    set with its seeds, summed).  Returns (terms dict, grad)."""
    pts = np.asarray(points, np.float64)
    sets = {"x": pts, "mx": mirror_points(pts, 1), "my": mirror_points(pts, 2), "ic": ic_points(ic_xy)}
    fg = {k: simulate(circ, params, v) for k, v in sets.items()}
    f, g = fg["x"]
    terms = total_loss(f, g, fg["mx"][0], fg["my"][0], fg["ic"][0], pts, ic_xy, desc)
    Vf, Wg, V_mx, V_my, V_ic = total_loss_seeds(f, g, fg["mx"][0], fg["my"][0], fg["ic"][0], pts, ic_xy, desc)
    grad = grad_reverse(circ, params, sets["x"], Vf, Wg)
    zero = lambda n: np.zeros((n, len(circ.out_qubits), 3))
    grad += grad_reverse(circ, params, sets["my"], V_my, zero(len(pts)))
    if desc.phys.kind == LOSS_VACUUM:
        grad += grad_reverse(circ, params, sets["mx"], V_mx, zero(len(pts)))
    if len(sets["ic"]):
        grad += grad_reverse(circ, params, sets["ic"], V_ic, zero(len(sets["ic"])))
    return terms, grad


# ---------------------------------------------------------------- diagnostics ------------------
# Section "'Black hole' loss landscape": the global Meyer-Wallach entanglement of the circuit's
# output state and the total field energy over time with its collapse indicator.

def reduced_density_matrices(psi, n):
    """rho_k [n, 2, 2] of one pure state psi [2^n] by explicit partial traces (qubit 0 = leftmost
    tensor factor): reshape to (2^k, 2, 2^(n-k-1)) and contract the other factors."""
    out = np.zeros((n, 2, 2), np.complex128)
    for k in range(n):
        t = psi.reshape(2 ** k, 2, 2 ** (n - k - 1))
        out[k] = np.einsum("aib,ajb->ij", t, np.conj(t))
    return out


def bloch_vectors(circ, params, points=None, angles=None, jac=None):
    """(<X_k>, <Y_k>, <Z_k>) [P, n, 3] of every qubit of every point's output state, from the reduced
    density matrices: rho = (I + r . sigma) / 2, so r = (2 Re rho_01, -2 Im rho_01, rho_00 - rho_11)."""
    psi, _ = final_states(circ, params, points, angles, jac)
    n, P = circ.n, psi.shape[1]
    r = np.zeros((P, n, 3))
    for p in range(P):
        rho = reduced_density_matrices(psi[:, p], n)
        r[p, :, 0] = 2 * rho[:, 0, 1].real
        r[p, :, 1] = -2 * rho[:, 0, 1].imag
        r[p, :, 2] = (rho[:, 0, 0] - rho[:, 1, 1]).real
    return r


def meyer_wallach(circ, params, points=None, angles=None, jac=None):
    """Global entanglement Q = 2 (1 - (1/n) sum_k Tr rho_k^2) of every point's output state
    (Meyer and Wallach's measure in Brennen's form): 0 for product states, 1 for GHZ states."""
    psi, _ = final_states(circ, params, points, angles, jac)
    n, P = circ.n, psi.shape[1]
    q = np.zeros(P)
    for p in range(P):
        rho = reduced_density_matrices(psi[:, p], n)
        purity = np.einsum("kij,kji->k", rho, rho).real
        q[p] = 2.0 * (1.0 - purity.mean())
    return q


def energy_grid(t_values, xg, yg):
    """Points (t, x, y) of the time slices t over the spatial grid xg x yg, t-major."""
    T, X, Y = np.meshgrid(np.asarray(t_values, np.float64), np.asarray(xg, np.float64),
                          np.asarray(yg, np.float64), indexing="ij")
    return np.stack([T.ravel(), X.ravel(), Y.ravel()], 1)


def energy_from_fields(f, points, n_t, desc):
    """U(t) = sum over the spatial grid of (eps E^2 + Hx^2 + Hy^2) / 2 for every time slice (f and
    points t-major, n_t slices)."""
    eps = _eps(points, desc)
    u = 0.5 * (eps * f[:, 0] ** 2 + f[:, 1] ** 2 + f[:, 2] ** 2)
    return u.reshape(n_t, -1).sum(axis=1)


def energy_profile(circ, params, t_values, xg, yg, desc):
    pts = energy_grid(t_values, xg, yg)
    f, _ = simulate(circ, params, pts)
    return energy_from_fields(f, pts, len(t_values), desc)


def black_hole_indicator(U, t_values, delta):
    """I_BH = 1 - min_{t in [delta, T]} U(t) / U(0) (U(0) the slice at t = 0)."""
    t = np.asarray(t_values, np.float64)
    U = np.asarray(U, np.float64)
    i0 = int(np.argmin(np.abs(t)))
    if t[i0] != 0.0:
        raise ValueError("the time slices must include t = 0")
    sel = t >= delta
    return float(1.0 - np.min(U[sel] / U[i0]))


# --------------------------------------------------------------- gradients --------------------

def grad_reverse(circ, params, points, seeds_f, seeds_g, angles=None, jac=None, chunk=None,
                 inputs=False):
    """d/dparams of  sum_p [ sum_i seeds_f[p,i] f_i + sum_ic seeds_g[p,i,c] g_ic ]  by plain
    stored-state reverse mode: every intermediate state is kept, the adjoints are pulled back
    through U^H, and each parametrised gate contributes
        2 Re [ <dU psi_in, lam_out> + sum_c <dU dpsi_c,in, mu_c,out> ].
    For the Maxwell loss pass seeds_f = 0 and seeds_g = maxwell_seeds(g).

    inputs=True (angle-given encoding only) also returns the derivatives of the same quantity
    with respect to the per-point angles [P,n] and Jacobian [P,n,3] (the inputs a classical
    layer in front of the circuit produces; section "QPINN architecture and ansatz designs",
    angle embedding): with lam_0, mu_c,0 the adjoints pulled back to the embedded product state,
        d/d theta_q = 2 Re [ <lam_0, d psi_0/d theta_q> + sum_c <mu_c,0, d dpsi_c,0/d theta_q> ],
        d/d J_qc    = 2 Re <mu_c,0, d dpsi_c,0/d J_qc>,
    where psi_0 = kron_q v(theta_q), dpsi_c,0 = sum_q J_qc kron(.., v'(theta_q), ..), so
    d dpsi_c,0/d J_qc = kron(.., v'(theta_q), ..) and d dpsi_c,0/d theta_q =
    sum_{q' != q} J_q'c kron(.., v'(theta_q'), .., v'(theta_q), ..) + J_qc kron(.., v''(theta_q), ..),
    all built by explicit Kronecker products per point."""
    params = np.asarray(params, np.float64)
    theta, J = encoding_angles(circ, points, angles, jac)
    ops = operators(circ, params)
    dops = operators(circ, params, derivative=True)
    n, P = circ.n, theta.shape[0]
    if chunk is None:   # bound the stored history to about 1 GB
        chunk = max(1, int(1e9 // (max(len(ops), 1) * 4 * 2 ** n * 16)))
    zd = [z_diagonal(n, i)[:, None] for i in circ.out_qubits]
    grad = np.zeros(circ.n_params)
    if inputs:
        if circ.enc.kind != ENC_ANGLES:
            raise ValueError("input gradients need the angle-given encoding")
        d_theta = np.zeros((P, n))
        d_J = np.zeros((P, n, 3))
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        psi, dpsi = initial_states(circ, theta[s:e], J[s:e])
        hist = []
        for U in ops:
            hist.append((psi, dpsi.copy()))
            psi = U @ psi
            dpsi = np.stack([U @ dpsi[c] for c in range(3)])
        Wf = np.asarray(seeds_f[s:e]) if seeds_f is not None else np.zeros((e - s, len(zd)))
        Wg = np.asarray(seeds_g[s:e])
        lam = np.zeros_like(psi)
        mu = np.zeros_like(dpsi)
        for k, z in enumerate(zd):
            lam += z * psi * Wf[None, :, k]
            for c in range(3):
                lam += z * dpsi[c] * Wg[None, :, k, c]
                mu[c] += z * psi * Wg[None, :, k, c]
        for idx in range(len(ops) - 1, -1, -1):
            psi_in, dpsi_in = hist[idx]
            kind, q0, q1, pi = circ.gates[idx]
            if pi >= 0:
                dU = dops[idx]
                acc = np.sum(np.conj(dU @ psi_in) * lam)
                for c in range(3):
                    acc += np.sum(np.conj(dU @ dpsi_in[c]) * mu[c])
                grad[pi] += 2.0 * np.real(acc)
            UH = ops[idx].conj().T
            lam = UH @ lam
            mu = np.stack([UH @ mu[c] for c in range(3)])
        if inputs:
            _input_grads(circ, theta[s:e], J[s:e], lam, mu, d_theta[s:e], d_J[s:e])
    if inputs:
        return grad, d_theta, d_J
    return grad


def _input_grads(circ, theta, J, lam, mu, d_theta, d_J):
    """Fills d_theta [P,n] and d_J [P,n,3] from the adjoints lam [2^n,P], mu [3,2^n,P] at the
    embedded product state (see grad_reverse)."""
    P, n = theta.shape
    v, dv = _embed_vectors(circ.enc.gate, theta)
    d2v = _embed_second_derivative(circ.enc.gate, theta)
    for p in range(P):
        for q in range(n):
            # d psi_0 / d theta_q and d dpsi_c,0 / d J_qc: v'(theta_q) in slot q
            t_q = _kron_list([dv[p, qq] if qq == q else v[p, qq] for qq in range(n)], False)
            acc = np.vdot(lam[:, p], t_q)
            for c in range(3):
                d_J[p, q, c] = 2.0 * np.real(np.vdot(mu[c, :, p], t_q))
                dd = J[p, q, c] * _kron_list([d2v[p, qq] if qq == q else v[p, qq] for qq in range(n)], False)
                for q2 in range(n):
                    if q2 != q and J[p, q2, c] != 0.0:
                        dd = dd + J[p, q2, c] * _kron_list(
                            [dv[p, qq] if qq in (q, q2) else v[p, qq] for qq in range(n)], False)
                acc += np.vdot(mu[c, :, p], dd)
            d_theta[p, q] = 2.0 * np.real(acc)


def maxwell_eval(circ, params, points, desc, angles=None, jac=None):
    """Everything the fused hot path returns: f, g, loss and d loss / d params (reverse mode)."""
    f, g = simulate(circ, params, points, angles, jac)
    loss = maxwell_loss(g, points, desc)
    W = maxwell_seeds(g, points, desc)
    grad = grad_reverse(circ, params, points, None, W, angles, jac)
    return f, g, loss, grad


def _shifted(circ, params, k, delta, points, angles, jac):
    p = params.copy()
    p[k] += delta
    return simulate(circ, p, points, angles, jac)


def grad_param_shift(circ, params, points, seeds_f, seeds_g, angles=None, jac=None):
    """Same quantity as grad_reverse, by parameter-shift rules applied to f and g, then
    contracted with the (fixed) seeds.  Valid when each parameter drives gates of one kind.

    Rotations exp(-i theta P/2) (generator eigenvalues +-1/2, one frequency):
        d f / d theta = [f(theta + pi/2) - f(theta - pi/2)] / 2.
    CRZ (generator |1><1| (x) Z/2, eigenvalues 0, 0, +-1/2: frequencies 1/2 and 1), the
    four-term rule of the general parameter-shift literature:
        d f / d theta = c1 [f(theta + pi/2) - f(theta - pi/2)] - c2 [f(theta + 3pi/2) - f(theta - 3pi/2)],
        c1 = (sqrt2 + 1) / (4 sqrt2),  c2 = (sqrt2 - 1) / (4 sqrt2).
    (The two-term rule is wrong for CRZ: it does not cancel the frequency-1/2 term.)"""
    params = np.asarray(params, np.float64)
    grad = np.zeros(circ.n_params)
    kinds = {}
    for kind, q0, q1, pi in circ.gates:
        if pi >= 0:
            kinds.setdefault(pi, set()).add(kind == CRZ)
    c1 = (math.sqrt(2.0) + 1.0) / (4.0 * math.sqrt(2.0))
    c2 = (math.sqrt(2.0) - 1.0) / (4.0 * math.sqrt(2.0))
    for k in range(circ.n_params):
        ks = kinds.get(k, set())
        if len(ks) > 1:
            raise ValueError(f"parameter {k} drives both rotations and CRZ gates")
        fp, gp = _shifted(circ, params, k, math.pi / 2, points, angles, jac)
        fm, gm = _shifted(circ, params, k, -math.pi / 2, points, angles, jac)
        if ks == {True}:
            fp3, gp3 = _shifted(circ, params, k, 3 * math.pi / 2, points, angles, jac)
            fm3, gm3 = _shifted(circ, params, k, -3 * math.pi / 2, points, angles, jac)
            df = c1 * (fp - fm) - c2 * (fp3 - fm3)
            dg = c1 * (gp - gm) - c2 * (gp3 - gm3)
        else:
            df, dg = (fp - fm) / 2.0, (gp - gm) / 2.0
        grad[k] = np.sum(dg * seeds_g)
        if seeds_f is not None:
            grad[k] += np.sum(df * seeds_f)
    return grad


def input_grads_param_shift(circ, params, seeds_f, seeds_g, angles, jac):
    """The input derivatives of grad_reverse(..., inputs=True) by the embedding's shift rule,
    forward simulations only.  Each angle theta_q enters one rotation exp(-i theta P/2), so
      d f_i / d theta_q = [f_i(theta_q + pi/2) - f_i(theta_q - pi/2)] / 2,
      d^2 f_i / d theta_q d theta_q' = [f(++) - f(+-) - f(-+) + f(--)] / 4          (q != q'),
      d^2 f_i / d theta_q^2 = [f(theta_q + pi) - f(theta_q)] / 2,
    and the tangents are g_ic = sum_q J_qc d f_i / d theta_q, so
      d/d J_qc     = sum_i seeds_g[i,c] d f_i / d theta_q,
      d/d theta_q  = sum_i seeds_f[i] d f_i / d theta_q
                     + sum_ic seeds_g[i,c] sum_q' J_q'c d^2 f_i / d theta_q d theta_q'."""
    if circ.enc.kind != ENC_ANGLES:
        raise ValueError("input gradients need the angle-given encoding")
    th = np.asarray(angles, np.float64)
    J = np.asarray(jac, np.float64)
    P, n = th.shape
    zeros = np.zeros((P, n, 3))

    def f_at(shifts):
        t = th.copy()
        for q, d in shifts:
            t[:, q] += d
        return simulate(circ, params, None, t, zeros)[0]      # [P, m]

    h = math.pi / 2
    f0 = f_at([])
    df = np.stack([(f_at([(q, h)]) - f_at([(q, -h)])) / 2.0 for q in range(n)], 1)    # [P,n,m]
    d2f = np.zeros((P, n, n, f0.shape[1]))
    for q in range(n):
        d2f[:, q, q] = (f_at([(q, math.pi)]) - f0) / 2.0
        for q2 in range(q + 1, n):
            v = (f_at([(q, h), (q2, h)]) - f_at([(q, h), (q2, -h)])
                 - f_at([(q, -h), (q2, h)]) + f_at([(q, -h), (q2, -h)])) / 4.0
            d2f[:, q, q2] = v
            d2f[:, q2, q] = v
    Wg = np.asarray(seeds_g, np.float64)                       # [P,m,3]
    d_J = np.einsum("pqi,pic->pqc", df, Wg)
    dg = np.einsum("pqri,prc->pqic", d2f, J)                   # d g_ic / d theta_q
    d_theta = np.einsum("pqic,pic->pq", dg, Wg)
    if seeds_f is not None:
        d_theta += np.einsum("pqi,pi->pq", df, np.asarray(seeds_f, np.float64))
    return d_theta, d_J


def grad_fd_loss(circ, params, points, desc, h=1e-6, idx=None, angles=None, jac=None):
    """Central finite differences of the Maxwell loss itself."""
    params = np.asarray(params, np.float64)
    idx = range(circ.n_params) if idx is None else idx
    out = {}
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        _, gp = simulate(circ, pp, points, angles, jac)
        _, gm = simulate(circ, pm, points, angles, jac)
        out[k] = (maxwell_loss(gp, points, desc) - maxwell_loss(gm, points, desc)) / (2 * h)
    return out


def fd_tangents(circ, params, points, h=1e-5):
    """Central finite differences of f in each input coordinate (the plain method's tangents)."""
    pts = np.asarray(points, np.float64)
    out = np.zeros((pts.shape[0], len(circ.out_qubits), 3))
    for c in range(3):
        pp, pm = pts.copy(), pts.copy()
        pp[:, c] += h
        pm[:, c] -= h
        fp, _ = simulate(circ, params, pp)
        fm, _ = simulate(circ, params, pm)
        out[:, :, c] = (fp - fm) / (2 * h)
    return out


def encoding_shift_tangents(circ, params, points):
    """Input tangents through the encoding's own parameter-shift rule: each embedded angle
    theta_q enters one rotation, so d f / d theta_q = [f(theta_q + pi/2) - f(theta_q - pi/2)]/2
    exactly, and d f / d c = sum_q J_qc d f / d theta_q."""
    theta, J = encoding_angles(circ, points)
    P, n = theta.shape
    zeros = np.zeros((P, n, 3))
    out = np.zeros((P, len(circ.out_qubits), 3))
    from copy import copy
    c_ang = copy(circ)
    c_ang.enc = copy(circ.enc)
    c_ang.enc.kind = ENC_ANGLES
    for q in range(n):
        tp, tm = theta.copy(), theta.copy()
        tp[:, q] += math.pi / 2
        tm[:, q] -= math.pi / 2
        fp, _ = simulate(c_ang, params, points, tp, zeros)
        fm, _ = simulate(c_ang, params, points, tm, zeros)
        d = (fp - fm) / 2.0
        out += d[:, :, None] * J[:, q, None, :]
    return out


def unitary(circ, params):
    """Dense product V = U_F ... U_1 of the full operators (brute force; small n only)."""
    V = np.eye(2 ** circ.n, dtype=np.complex128)
    for U in operators(circ, np.asarray(params, np.float64)):
        V = (U @ V) if not sp.issparse(U) else U @ V
    return V
