"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test checks the oracle against something other than itself: closed forms, Bloch-sphere
geometry, Bell/GHZ states, an independent bit-level simulator built on scipy's expm, the trace
identity of the Z readout, the parameter-shift rule, finite differences, an exact plane-wave
solution of the TE_z system, and the parameter counts printed in the paper's Table 1.
"""
import json
import math
import os
from copy import deepcopy

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import qpinn_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _circ(n, gates, n_params, enc=None, out=None):
    return W.Circuit(n=n, gates=gates, n_params=n_params, enc=enc or W.Encoding(),
                     out_qubits=out if out is not None else list(range(min(n, 3))))


# ------------------------------------------------------------------ closed forms --------------

def test_ry_embedding_closed_form():
    """<Z> = cos(theta) after RY(theta)|0>; cycled pi-scaling gives theta = pi*c, so
    <Z_q> = cos(pi c) and d<Z_q>/dc = -pi sin(pi c) on the qubit's own coordinate only."""
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 1, (17, 3))
    c = _circ(5, [], 0, out=[0, 1, 2, 3, 4])
    f, g = O.simulate(c, [], pts)
    for q in range(5):
        col = q % 3
        np.testing.assert_allclose(f[:, q], np.cos(math.pi * pts[:, col]), atol=1e-14)
        for cc in range(3):
            exp = -math.pi * np.sin(math.pi * pts[:, col]) if cc == col else 0.0
            np.testing.assert_allclose(g[:, q, cc], exp, atol=1e-13)


def test_rx_scaling_identities_golden():
    """Caption of the input-scaling figure: RX(arccos a) gives <Z> = a, RX(arcsin a + pi/2)
    gives <Z> = -a."""
    gold = json.load(open(os.path.join(GOLDEN, "scaling_identities.json")))
    a = np.array(gold["a"])
    pts = np.stack([a, np.zeros_like(a), np.zeros_like(a)], 1)
    for scale, key in ((W.SCALE_ACOS, "acos_expect_z"), (W.SCALE_ASIN, "asin_expect_z")):
        enc = W.Encoding(kind=W.ENC_CYCLE, gate=W.ENC_RX, scale=scale, coord_of_qubit=[0])
        with np.errstate(divide="ignore", invalid="ignore"):
            f, _ = O.simulate(_circ(1, [], 0, enc=enc, out=[0]), [], pts)
        np.testing.assert_allclose(f[:, 0], gold[key], atol=1e-12)


def test_rx_embedding_phase_closed_form():
    """The RX embedding is exp(-i theta X/2)|0>, so a following RX(pi/2) turns it into
    RX(theta + pi/2)|0> with <Z> = cos(theta + pi/2) = -sin(theta) (theta = pi t here); the
    opposite phase, exp(+i theta X/2)|0>, would give +sin(theta) though <Z> alone cannot tell."""
    t = np.linspace(-0.95, 0.95, 9)
    pts = np.stack([t, np.zeros_like(t), np.zeros_like(t)], 1)
    enc = W.Encoding(kind=W.ENC_CYCLE, gate=W.ENC_RX, scale=W.SCALE_PI, coord_of_qubit=[0])
    circ = _circ(1, [(W.RX, 0, -1, 0)], 1, enc=enc, out=[0])
    f, g = O.simulate(circ, [math.pi / 2], pts)
    np.testing.assert_allclose(f[:, 0], -np.sin(math.pi * t), atol=1e-14)
    np.testing.assert_allclose(g[:, 0, 0], -math.pi * np.cos(math.pi * t), atol=1e-13)
    np.testing.assert_allclose(g[:, 0, 1:], 0.0, atol=1e-15)


def test_scale_derivatives_match_finite_differences():
    a = np.linspace(-0.9, 0.9, 11)
    h = 1e-6
    for s in range(5):
        fd = (O.scale_value(s, a + h) - O.scale_value(s, a - h)) / (2 * h)
        np.testing.assert_allclose(O.scale_derivative(s, a), fd, rtol=1e-8, atol=1e-9)


# ------------------------------------------------------------- Bloch-sphere pin ---------------

def _so3(kind, phi):
    c, s = math.cos(phi), math.sin(phi)
    if kind == W.RX:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if kind == W.RY:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _so3_d(kind, phi):
    c, s = math.cos(phi), math.sin(phi)
    if kind == W.RX:
        return np.array([[0, 0, 0], [0, -s, -c], [0, c, -s]])
    if kind == W.RY:
        return np.array([[-s, 0, c], [0, 0, 0], [-c, 0, -s]])
    return np.array([[-s, -c, 0], [c, -s, 0], [0, 0, 0]])


@pytest.mark.parametrize("rot,n,L", [("xyz", 3, 3), ("rot", 4, 2), ("xyz", 12, 2)])
def test_product_state_matches_bloch_rotations(rot, n, L):
    """With no entangler (the No-Entanglement ansatz) every qubit stays a product factor whose
    Bloch vector is turned by the SO(3) rotation of each gate; <Z> is its z component.  This
    pins outputs, input tangents and reverse-mode gradients at any n (here up to 12) without a
    statevector."""
    rng = np.random.default_rng(1)
    circ = W.no_entanglement(n, L, rot)
    circ.out_qubits = list(range(n))
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    pts = rng.uniform(-1, 1, (4, 3))
    f, g = O.simulate(circ, params, pts)
    seeds = rng.standard_normal(g.shape)
    seeds_f = rng.standard_normal(f.shape)
    grad = O.grad_reverse(circ, params, pts, seeds_f, seeds)
    exp_grad = np.zeros(circ.n_params)
    for p in range(pts.shape[0]):
        for q in range(n):
            th = math.pi * pts[p, q % 3]
            b0 = np.array([math.sin(th), 0.0, math.cos(th)])
            db0 = np.array([math.cos(th), 0.0, -math.sin(th)]) * math.pi
            ops = [(k, prm) for (k, qq, _, prm) in circ.gates if qq == q]
            Rs = [_so3(k, params[prm]) for k, prm in ops]
            b, db = b0.copy(), db0.copy()
            for R in Rs:
                b, db = R @ b, R @ db
            assert abs(f[p, q] - b[2]) < 1e-12
            for cc in range(3):
                exp = db[2] if cc == q % 3 else 0.0
                assert abs(g[p, q, cc] - exp) < 1e-12
            for i, (k, prm) in enumerate(ops):
                before = np.eye(3)
                for R in Rs[:i]:
                    before = R @ before
                after = np.eye(3)
                for R in Rs[i + 1:]:
                    after = R @ after
                D = after @ _so3_d(k, params[prm]) @ before
                exp_grad[prm] += seeds_f[p, q] * (D @ b0)[2]
                exp_grad[prm] += seeds[p, q, q % 3] * (D @ db0)[2]
    np.testing.assert_allclose(grad, exp_grad, atol=1e-11)


# ------------------------------------------------------------- entanglers ---------------------

def _zero_enc():
    return W.Encoding(kind=W.ENC_CYCLE, gate=W.ENC_RY, scale=W.SCALE_NONE)


def test_bell_state():
    """RY(pi/2) on qubit 0 then CNOT(0,1): amplitudes 1/sqrt2 on |00> and |11>, <Z0>=<Z1>=0."""
    circ = _circ(2, [(W.RY, 0, -1, 0), (W.CNOT, 0, 1, -1)], 1, enc=_zero_enc(), out=[0, 1])
    psi, _ = O.final_states(circ, [math.pi / 2], np.zeros((1, 3)))
    np.testing.assert_allclose(psi[:, 0], [2 ** -0.5, 0, 0, 2 ** -0.5], atol=1e-15)
    f, _ = O.simulate(circ, [math.pi / 2], np.zeros((1, 3)))
    np.testing.assert_allclose(f, 0.0, atol=1e-15)


def test_ghz_state_and_cnot_direction():
    n = 5
    gates = [(W.RY, 0, -1, 0)] + [(W.CNOT, q, q + 1, -1) for q in range(n - 1)]
    circ = _circ(n, gates, 1, enc=_zero_enc())
    psi, _ = O.final_states(circ, [math.pi / 2], np.zeros((1, 3)))
    exp = np.zeros(2 ** n)
    exp[0] = exp[-1] = 2 ** -0.5
    np.testing.assert_allclose(psi[:, 0], exp, atol=1e-15)
    # direction: control 0 (most significant bit), target 1.  |10> -> |11>, |01> -> |01>.
    circ = _circ(2, [(W.RY, 0, -1, 0), (W.CNOT, 0, 1, -1)], 1, enc=_zero_enc(), out=[0, 1])
    psi, _ = O.final_states(circ, [math.pi], np.zeros((1, 3)))
    np.testing.assert_allclose(np.abs(psi[:, 0]), [0, 0, 0, 1], atol=1e-15)
    circ = _circ(2, [(W.RY, 1, -1, 0), (W.CNOT, 0, 1, -1)], 1, enc=_zero_enc(), out=[0, 1])
    psi, _ = O.final_states(circ, [math.pi], np.zeros((1, 3)))
    np.testing.assert_allclose(np.abs(psi[:, 0]), [0, 1, 0, 0], atol=1e-15)


def _expm_rot(kind, th):
    P = {W.RX: np.array([[0, 1], [1, 0]]), W.RY: np.array([[0, -1j], [1j, 0]]),
         W.RZ: np.diag([1, -1])}[kind]
    return sla.expm(-0.5j * th * P)


def _bitwise_simulate(circ, params, psi0):
    """Independent simulator: loops over basis indices and flips bits (qubit 0 = MSB)."""
    n = circ.n
    s = np.array(psi0, dtype=np.complex128)
    for kind, q0, q1, pi in circ.gates:
        m0 = 1 << (n - 1 - q0)
        new = s.copy()
        if kind in (W.RX, W.RY, W.RZ):
            U = _expm_rot(kind, params[pi])
            for j in range(2 ** n):
                if j & m0:
                    continue
                a, b = s[j], s[j | m0]
                new[j] = U[0, 0] * a + U[0, 1] * b
                new[j | m0] = U[1, 0] * a + U[1, 1] * b
        else:
            m1 = 1 << (n - 1 - q1)
            for j in range(2 ** n):
                if not j & m0:
                    continue
                if kind == W.CNOT:
                    new[j] = s[j ^ m1]
                elif kind == W.CZ:
                    new[j] = -s[j] if j & m1 else s[j]
                elif kind == W.CRZ:
                    ph = np.exp(0.5j * params[pi]) if j & m1 else np.exp(-0.5j * params[pi])
                    new[j] = ph * s[j]
        s = new
    return s


@pytest.mark.parametrize("seed", range(4))
def test_kron_oracle_matches_bitwise_simulator(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 5))
    gates, K = [], 0
    for _ in range(14):
        k = int(rng.integers(0, 6))
        if k <= 2:
            gates.append((k, int(rng.integers(0, n)), -1, K))
            K += 1
        else:
            a, b = rng.choice(n, 2, replace=False)
            if k == W.CRZ:
                gates.append((k, int(a), int(b), K))
                K += 1
            else:
                gates.append((k, int(a), int(b), -1))
    params = rng.uniform(0, 2 * math.pi, K)
    circ = _circ(n, gates, K, out=list(range(n)))
    pts = rng.uniform(-1, 1, (3, 3))
    psi, dpsi = O.final_states(circ, params, pts)
    psi0, _ = O.initial_states(circ, *O.encoding_angles(circ, pts))
    for p in range(3):
        np.testing.assert_allclose(psi[:, p], _bitwise_simulate(circ, params, psi0[:, p]),
                                   atol=1e-13)
    # brute-force dense product of the full operators: unitary, and the same final state
    V = O.unitary(circ, params)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(2 ** n), atol=1e-12)
    np.testing.assert_allclose(V @ psi0, psi, atol=1e-13)


def test_cz_stride_ring_sign_function():
    """A CZ ring of stride r is the diagonal sign (-1)^(sum_q b_q b_(q+r mod n))."""
    for n, r in ((4, 1), (5, 2), (6, 3), (4, 2)):
        gates = W.ring(n, W.CZ, r)
        V = O.unitary(_circ(n, gates, 0), [])
        for j in range(2 ** n):
            bits = [(j >> (n - 1 - q)) & 1 for q in range(n)]
            e = sum(bits[q] * bits[(q + r) % n] for q in range(n) if (q + r) % n != q)
            assert V[j, j] == pytest.approx((-1) ** e)
        assert np.count_nonzero(V - np.diag(np.diag(V))) == 0


def test_operators_unitary_and_norm_preserved():
    w = W.config(1, P=8)
    ops = O.operators(w.circuit, w.params)
    for U in ops:
        np.testing.assert_allclose(U.conj().T @ U, np.eye(U.shape[0]), atol=1e-13)
    psi, _ = O.final_states(w.circuit, w.params, w.points)
    np.testing.assert_allclose(np.linalg.norm(psi, axis=0), 1.0, atol=1e-13)


def test_init_zeros_gives_unit_outputs():
    """Section on parameter initialisation: all-zero parameters without an embedding rotation
    give every output equal to 1 (here the embedding angle is 0 at the origin)."""
    for circ in (W.config(1, P=1).circuit, W.strongly_entangling(5, 3, ent=W.CZ)):
        circ = deepcopy(circ)
        circ.out_qubits = list(range(circ.n))
        f, g = O.simulate(circ, np.zeros(circ.n_params), np.zeros((2, 3)))
        np.testing.assert_allclose(f, 1.0, atol=1e-14)
        np.testing.assert_allclose(g, 0.0, atol=1e-14)


def test_trace_identity_over_basis_encodings():
    """Summing <Z_i> over all 2^n basis-state inputs gives Tr(V^H Z_i V) = Tr(Z_i) = 0, the
    discrete form of the zero-mean statement in the initialisation section."""
    rng = np.random.default_rng(3)
    for circ in (W.basic_entangling(4, 3, "xyz"), W.strongly_entangling(5, 2, ent=W.CZ)):
        circ = deepcopy(circ)
        circ.out_qubits = list(range(circ.n))
        circ.enc = W.Encoding(kind=W.ENC_ANGLES)
        n = circ.n
        theta = np.array([[math.pi * ((j >> (n - 1 - q)) & 1) for q in range(n)]
                          for j in range(2 ** n)])
        params = rng.uniform(0, 2 * math.pi, circ.n_params)
        f, _ = O.simulate(circ, params, np.zeros((2 ** n, 3)), theta, np.zeros((2 ** n, n, 3)))
        np.testing.assert_allclose(f.sum(0), 0.0, atol=1e-12)
        assert np.abs(f).max() > 0.05


# ------------------------------------------------------------ derivatives ---------------------

def _small(k, P):
    w = W.config(k, P=P)
    if k == 0:
        w.loss = W.MaxwellDesc(W.LOSS_VACUUM)
    return w


@pytest.mark.parametrize("k", [1, 2])
def test_tangents_match_fd_and_encoding_shift(k):
    w = _small(k, 6)
    _, g = O.simulate(w.circuit, w.params, w.points)
    fd = O.fd_tangents(w.circuit, w.params, w.points, h=1e-5)
    np.testing.assert_allclose(g, fd, atol=2e-8 if k == 1 else 5e-8)
    if w.circuit.enc.kind == W.ENC_CYCLE:
        sh = O.encoding_shift_tangents(w.circuit, w.params, w.points)
        np.testing.assert_allclose(g, sh, atol=1e-12)


def test_rff_jacobian_matches_fd():
    w = W.config(2, P=5)
    th, J = O.encoding_angles(w.circuit, w.points)
    h = 1e-6
    for c in range(3):
        pp, pm = w.points.astype(np.float64), w.points.astype(np.float64)
        pp = pp.copy(); pm = pm.copy()
        pp[:, c] += h
        pm[:, c] -= h
        fd = (O.encoding_angles(w.circuit, pp)[0] - O.encoding_angles(w.circuit, pm)[0]) / (2 * h)
        np.testing.assert_allclose(J[:, :, c], fd, atol=1e-8)


@pytest.mark.parametrize("name", ["c2", "c3", "mixed"])
def test_reverse_mode_equals_parameter_shift(name):
    if name == "c2":
        w = _small(1, 5)
    elif name == "c3":
        w = W.config(2, P=6)
        w.circuit = deepcopy(w.circuit)
        w.circuit.gates = [g for g in w.circuit.gates if g[3] < 48 or g[3] < 0][:]
        # keep the first two layers (48 params) and their rings
        keep, K = [], 0
        for g in W.config(2, P=1).circuit.gates:
            if g[3] >= 48:
                break
            keep.append(g)
        w.circuit.gates, w.circuit.n_params = keep, 48
        w.params = w.params[:48]
    else:
        b = W.batch_config(P_cap=5)
        w = min(b, key=lambda x: x.circuit.n_params)
    f, g = O.simulate(w.circuit, w.params, w.points)
    seeds = O.maxwell_seeds(g, w.points, w.loss)
    rev = O.grad_reverse(w.circuit, w.params, w.points, None, seeds)
    sh = O.grad_param_shift(w.circuit, w.params, w.points, None, seeds)
    np.testing.assert_allclose(rev, sh, atol=1e-12 * max(1, np.abs(sh).max()))


def test_reverse_mode_matches_fd_of_loss():
    w = W.config(2, P=8)
    f, g, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    fd = O.grad_fd_loss(w.circuit, w.params, w.points, w.loss, h=1e-5, idx=[0, 7, 100, 233])
    for k, v in fd.items():
        assert abs(v - grad[k]) <= 1e-7 * max(1.0, abs(grad[k])), (k, v, grad[k])


def test_last_layer_diagonal_gradients_vanish():
    """A trailing Z rotation followed only by entangling permutations/diagonals cannot change
    Z-basis probabilities: its gradient is exactly zero (last-layer RZ; last-layer Rot omega)."""
    for k in (1, 2):
        w = W.config(k, P=4)
        _, _, _, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
        n = w.circuit.n
        K = w.circuit.n_params
        last = [K - 3 * n + 3 * q + 2 for q in range(n)]
        assert np.abs(grad[last]).max() < 1e-14
        assert np.abs(grad).max() > 1e-3


def test_two_pi_periodicity():
    """theta -> theta + 2 pi flips the sign of the state: outputs, tangents, gradients unchanged."""
    w = _small(1, 4)
    f, g, L, gr = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    p2 = w.params.astype(np.float64).copy()
    p2[[3, 17, 50]] += 2 * math.pi
    f2, g2, L2, gr2 = O.maxwell_eval(w.circuit, p2, w.points, w.loss)
    np.testing.assert_allclose(f2, f, atol=1e-13)
    np.testing.assert_allclose(g2, g, atol=1e-12)
    np.testing.assert_allclose(gr2, gr, atol=1e-12)


# ------------------------------------------------------------------ loss ----------------------

def _wave(points, eps_of_point, sign=-1.0):
    """g for E = F(x - v t), Hx = 0, Hy = sign * sqrt(eps) F(x - v t), v = 1/sqrt(eps),
    with F(s) = exp(-s^2) sin(3 s)."""
    t, x = points[:, 0], points[:, 1]
    v = 1.0 / np.sqrt(eps_of_point)
    s = x - v * t
    Fp = np.exp(-s * s) * (3 * np.cos(3 * s) - 2 * s * np.sin(3 * s))
    g = np.zeros((points.shape[0], 3, 3))
    g[:, 0, 0] = -v * Fp
    g[:, 0, 1] = Fp
    a = sign * np.sqrt(eps_of_point)
    g[:, 2, 0] = -a * v * Fp
    g[:, 2, 1] = a * Fp
    return g, Fp


def test_plane_wave_is_an_exact_zero_of_every_residual():
    """E_z = F(x - t/sqrt(eps)), H_y = -sqrt(eps) F(...), H_x = 0 solves the TE_z system with
    permittivity eps, so every residual, the loss and all seeds vanish; flipping H_y gives
    r1 = r3 = -2F' (vacuum): loss = 8 mean(F'^2)."""
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1, 1, (64, 3))
    g, _ = _wave(pts, np.ones(64))
    d = W.MaxwellDesc(W.LOSS_VACUUM)
    assert O.maxwell_loss(g, pts, d) < 1e-28
    assert np.abs(O.maxwell_seeds(g, pts, d)).max() < 1e-14
    for kind in (W.LOSS_DIEL_SPLIT, W.LOSS_DIEL_INTUITIVE):
        d = W.MaxwellDesc(kind, eps_r=4.0)
        eps = np.where(pts[:, 1] >= 0, 4.0, 1.0)
        g, _ = _wave(pts, eps)
        assert O.maxwell_loss(g, pts, d) < 1e-28
    g, Fp = _wave(pts, np.ones(64), sign=+1.0)
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_VACUUM)) == pytest.approx(
        8 * np.mean(Fp ** 2), rel=1e-12)


def test_dielectric_split_weights():
    """Split loss (eq. phys_loss_diel): MSE over the vacuum half plus MSE over the dielectric
    half.  dE/dt = 1 everywhere gives r1 = 1: split = 2, intuitive = vacuum = 1.  dHy/dx = 1
    gives r1 = -1/eps: split = 1 + 1/16, intuitive = (N_vac + N_diel/16)/P."""
    rng = np.random.default_rng(6)
    pts = rng.uniform(-1, 1, (50, 3))
    nd = int((pts[:, 1] >= 0).sum())
    nv = 50 - nd
    g = np.zeros((50, 3, 3))
    g[:, 0, 0] = 1.0
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT)) == pytest.approx(2.0)
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_INTUITIVE)) == pytest.approx(1.0)
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_VACUUM)) == pytest.approx(1.0)
    g = np.zeros((50, 3, 3))
    g[:, 2, 1] = 1.0
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT)) == pytest.approx(1 + 1 / 16)
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_INTUITIVE)) == pytest.approx(
        (nv + nd / 16) / 50)


def test_split_loss_with_one_region_empty():
    """With every point in vacuum the split loss is the vacuum loss; with every point in the
    dielectric it is the intuitive form (eps_r everywhere, one mean over all points): the empty
    region's mean contributes nothing."""
    rng = np.random.default_rng(9)
    pts = rng.uniform(-1, 1, (40, 3))
    g = rng.standard_normal((40, 3, 3))
    vac = O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_VACUUM))
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=2.0)) == pytest.approx(vac)
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=-2.0)) == pytest.approx(
        O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_INTUITIVE, eps_r=4.0, x_interface=-2.0)))
    assert O.maxwell_loss(g, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT, eps_r=4.0, x_interface=-2.0)) != pytest.approx(vac)


def test_seeds_are_the_gradient_of_the_loss_in_g():
    rng = np.random.default_rng(7)
    pts = rng.uniform(-1, 1, (9, 3))
    g = rng.standard_normal((9, 3, 3))
    for kind in (W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT, W.LOSS_DIEL_INTUITIVE):
        d = W.MaxwellDesc(kind)
        S = O.maxwell_seeds(g, pts, d)
        h = 1e-6
        for idx in [(0, 0, 0), (3, 2, 1), (5, 1, 2), (8, 0, 2), (2, 0, 1), (4, 1, 0)]:
            gp, gm = g.copy(), g.copy()
            gp[idx] += h
            gm[idx] -= h
            fd = (O.maxwell_loss(gp, pts, d) - O.maxwell_loss(gm, pts, d)) / (2 * h)
            assert fd == pytest.approx(S[idx], abs=1e-8)


# ------------------------------------------------------------------ Table 1 -------------------

def test_table1_parameter_counts_golden():
    gold = json.load(open(os.path.join(GOLDEN, "table1_param_counts.json")))
    for name, count in gold["quantum_params"].items():
        c = W.paper_context_circuit(name, gold["n_qubits"], gold["n_layers"])
        assert c.n_params == count, name


# ------------------------------------------------- bias / none scalings, RFF angles, CRZ --------

@pytest.mark.parametrize("gate", [W.ENC_RY, W.ENC_RX])
def test_bias_and_none_scalings_closed_form_golden(gate):
    """Eq. scale's bias scaling (a + 1) pi/2 and the unscaled embedding: <Z> and d<Z>/da against
    closed forms written as other trig functions (-sin(pi a/2) and cos a), not the oracle's
    formula; both embedding gates give <Z> = cos(theta)."""
    gold = json.load(open(os.path.join(GOLDEN, "scaling_identities.json")))
    a = np.array(gold["a"])
    pts = np.stack([a, np.zeros_like(a), np.zeros_like(a)], 1)
    for scale, kz, kd in ((W.SCALE_BIAS, "bias_expect_z", "bias_dz_da"),
                          (W.SCALE_NONE, "none_expect_z", "none_dz_da")):
        enc = W.Encoding(kind=W.ENC_CYCLE, gate=gate, scale=scale, coord_of_qubit=[0])
        f, g = O.simulate(_circ(1, [], 0, enc=enc, out=[0]), [], pts)
        np.testing.assert_allclose(f[:, 0], gold[kz], atol=1e-14)
        np.testing.assert_allclose(g[:, 0, 0], gold[kd], atol=1e-13)
        np.testing.assert_allclose(g[:, 0, 1:], 0.0, atol=1e-15)


def test_rff_angles_one_frequency_closed_form():
    """Random Fourier features with one frequency b and a map W that picks one slot per qubit:
    theta_0 = 0.5 cos(b.p), theta_1 = 2 sin(b.p) (no 2 pi, cosine half first).  With the RY
    embedding <Z_q> = cos(theta_q) and d<Z_q>/dc = -sin(theta_q) d theta_q/dc, where
    d cos(b.p)/dc = -sin(b.p) b_c and d sin(b.p)/dc = cos(b.p) b_c."""
    b = np.array([0.7, -1.3, 0.4])
    Wm = np.array([[0.5, 0.0], [0.0, 2.0]])
    enc = W.Encoding(kind=W.ENC_RFF, gate=W.ENC_RY, scale=W.SCALE_NONE, rff_B=b[None, :], rff_W=Wm)
    rng = np.random.default_rng(11)
    pts = rng.uniform(-1, 1, (9, 3))
    f, g = O.simulate(_circ(2, [], 0, enc=enc, out=[0, 1]), [], pts)
    bp = pts @ b
    th0, th1 = 0.5 * np.cos(bp), 2.0 * np.sin(bp)
    np.testing.assert_allclose(f[:, 0], np.cos(th0), atol=1e-14)
    np.testing.assert_allclose(f[:, 1], np.cos(th1), atol=1e-14)
    for c in range(3):
        np.testing.assert_allclose(g[:, 0, c], -np.sin(th0) * (-0.5 * np.sin(bp) * b[c]), atol=1e-13)
        np.testing.assert_allclose(g[:, 1, c], -np.sin(th1) * (2.0 * np.cos(bp) * b[c]), atol=1e-13)


def _cross_mesh_small():
    """3-qubit, 2-layer Cross-Mesh circuit (RX per qubit, CRZ on every ordered pair; eq.
    crz_cross_mesh) with random parameters and points, vacuum Maxwell loss."""
    circ = W.cross_mesh(3, 2, "xz", W.CRZ)
    rng = np.random.default_rng(21)
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    pts = rng.uniform(-1, 1, (4, 3))
    return circ, params, pts, W.MaxwellDesc(W.LOSS_VACUUM)


def test_crz_gradient_matches_fd_of_loss():
    """The CRZ derivative branch and the reverse sweep through CRZ against central finite
    differences of the loss (which use only the forward operators)."""
    circ, params, pts, loss = _cross_mesh_small()
    _, _, _, grad = O.maxwell_eval(circ, params, pts, loss)
    crz = sorted({g[3] for g in circ.gates if g[0] == W.CRZ})
    fd = O.grad_fd_loss(circ, params, pts, loss, h=1e-5, idx=crz[:6] + [0, 4])
    for k, v in fd.items():
        assert abs(v - grad[k]) <= 1e-8 * max(1.0, abs(grad[k])), (k, v, grad[k])
    assert np.abs(grad[crz]).max() > 1e-3


def test_crz_gradient_matches_four_term_shift_rule():
    """Reverse mode through CRZ against the four-term shift rule (generator eigenvalues 0,
    +-1/2), which is exact; the two-term rule is checked to be wrong for CRZ here."""
    circ, params, pts, loss = _cross_mesh_small()
    f, g = O.simulate(circ, params, pts)
    seeds = O.maxwell_seeds(g, pts, loss)
    rev = O.grad_reverse(circ, params, pts, None, seeds)
    sh = O.grad_param_shift(circ, params, pts, None, seeds)
    np.testing.assert_allclose(rev, sh, atol=1e-12 * max(1.0, np.abs(sh).max()))
    k = next(g[3] for g in circ.gates if g[0] == W.CRZ)
    fp, gp = O._shifted(circ, np.asarray(params, np.float64), k, math.pi / 2, pts, None, None)
    fm, gm = O._shifted(circ, np.asarray(params, np.float64), k, -math.pi / 2, pts, None, None)
    two_term = float(np.sum((gp - gm) / 2.0 * seeds))
    assert abs(two_term - rev[k]) > 1e-6 * max(1.0, abs(rev[k]))


def _angles_case(gate, seed=3, P=3, n=3, L=2):
    """A small angle-given circuit (RX or RY embedding, Rot + CNOT ring), random angles and a
    dense random Jacobian, and random VJP seeds."""
    rng = np.random.default_rng(seed)
    enc = W.Encoding(kind=W.ENC_ANGLES, gate=gate)
    circ = W.basic_entangling(n, L, "rot", enc=enc)
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    th = rng.uniform(-2.0, 2.0, (P, n))
    J = rng.standard_normal((P, n, 3))
    m = len(circ.out_qubits)
    return circ, params, th, J, rng.standard_normal((P, m)), rng.standard_normal((P, m, 3))


def _vjp_objective(circ, params, th, J, sf, sg):
    f, g = O.simulate(circ, params, None, th, J)
    return float(np.sum(sf * f) + np.sum(sg * g))


@pytest.mark.parametrize("gate", [W.ENC_RY, W.ENC_RX])
def test_input_gradients_match_fd(gate):
    """d/d(angles) and d/d(Jacobian) of reverse mode against central finite differences of the
    objective sum(seeds_f f) + sum(seeds_g g), which uses only the forward simulation."""
    circ, params, th, J, sf, sg = _angles_case(gate)
    _, d_th, d_J = O.grad_reverse(circ, params, None, sf, sg, th, J, inputs=True)
    h = 1e-6
    for p in range(th.shape[0]):
        for q in range(th.shape[1]):
            tp, tm = th.copy(), th.copy()
            tp[p, q] += h
            tm[p, q] -= h
            fd = (_vjp_objective(circ, params, tp, J, sf, sg) - _vjp_objective(circ, params, tm, J, sf, sg)) / (2 * h)
            assert abs(fd - d_th[p, q]) < 1e-8, (p, q, fd, d_th[p, q])
            for c in range(3):
                jp, jm = J.copy(), J.copy()
                jp[p, q, c] += h
                jm[p, q, c] -= h
                fd = (_vjp_objective(circ, params, th, jp, sf, sg) - _vjp_objective(circ, params, th, jm, sf, sg)) / (2 * h)
                assert abs(fd - d_J[p, q, c]) < 1e-8, (p, q, c, fd, d_J[p, q, c])


@pytest.mark.parametrize("gate", [W.ENC_RY, W.ENC_RX])
def test_input_gradients_match_embedding_shift_rule(gate):
    """Reverse mode against the embedding's exact shift rules (first and second derivatives of
    the readouts from shifted forward simulations)."""
    circ, params, th, J, sf, sg = _angles_case(gate, seed=5, P=4, n=4)
    _, d_th, d_J = O.grad_reverse(circ, params, None, sf, sg, th, J, inputs=True)
    s_th, s_J = O.input_grads_param_shift(circ, params, sf, sg, th, J)
    np.testing.assert_allclose(d_th, s_th, atol=1e-12)
    np.testing.assert_allclose(d_J, s_J, atol=1e-12)
    assert np.abs(d_th).max() > 1e-2 and np.abs(d_J).max() > 1e-2


def test_input_gradients_of_the_maxwell_loss_match_fd():
    """The Maxwell loss (quadratic in the tangents) through its seeds: reverse-mode input
    gradients against central finite differences of the loss itself."""
    circ, params, th, J, _, _ = _angles_case(W.ENC_RX, seed=9, P=4)
    pts = np.random.default_rng(2).uniform(-1, 1, (4, 3))
    desc = W.MaxwellDesc(W.LOSS_DIEL_SPLIT, 4.0, 0.0)

    def loss(t, j):
        return O.maxwell_loss(O.simulate(circ, params, pts, t, j)[1], pts, desc)
    _, g = O.simulate(circ, params, pts, th, J)
    _, d_th, d_J = O.grad_reverse(circ, params, pts, None, O.maxwell_seeds(g, pts, desc), th, J, inputs=True)
    h = 1e-6
    for (p, q) in [(0, 0), (1, 2), (3, 1)]:
        tp, tm = th.copy(), th.copy()
        tp[p, q] += h
        tm[p, q] -= h
        assert abs((loss(tp, J) - loss(tm, J)) / (2 * h) - d_th[p, q]) < 1e-8
        for c in range(3):
            jp, jm = J.copy(), J.copy()
            jp[p, q, c] += h
            jm[p, q, c] -= h
            assert abs((loss(th, jp) - loss(th, jm)) / (2 * h) - d_J[p, q, c]) < 1e-8


# ------------------------------------------------------------ the paper's total loss -----------

def _analytic_fields(pts, a=(1.3, -0.7, 0.4), b=(0.9, 1.1, -1.5)):
    """Smooth fields that solve nothing: E = sin(k.p), Hx = cos(l.p), Hy = sin(k.p) cos(l.p), with
    their exact derivatives (p = (t, x, y))."""
    k, l = np.array(a), np.array(b)
    sk, ck = np.sin(pts @ k), np.cos(pts @ k)
    sl, cl = np.sin(pts @ l), np.cos(pts @ l)
    f = np.stack([sk, cl, sk * cl], 1)
    g = np.zeros((len(pts), 3, 3))
    g[:, 0, :] = ck[:, None] * k
    g[:, 1, :] = -sl[:, None] * l
    g[:, 2, :] = (ck * cl)[:, None] * k - (sk * sl)[:, None] * l
    return f, g


@pytest.mark.parametrize("kind", [W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT])
def test_energy_residual_is_the_poynting_balance(kind):
    """e = du/dt + dSx/dx + dSy/dy with u = (eps E^2 + Hx^2 + Hy^2)/2, S = (-E Hy, E Hx) (the
    Poynting theorem with J = 0), checked by central differences of u and S on analytic fields;
    and the vacuum plane wave (E, Hx, Hy) = (F(x - t), 0, -F(x - t)) has e = 0."""
    rng = np.random.default_rng(11)
    pts = rng.uniform(-1, 1, (16, 3))
    desc = W.MaxwellDesc(kind, 4.0, 0.0)
    f, g = _analytic_fields(pts)
    e = O.energy_residual(f, g, pts, desc)
    eps = np.where(pts[:, 1] >= 0, 4.0, 1.0) if kind != W.LOSS_VACUUM else np.ones(16)

    def u_s(p):
        ff, _ = _analytic_fields(p)
        return 0.5 * (eps * ff[:, 0] ** 2 + ff[:, 1] ** 2 + ff[:, 2] ** 2), -ff[:, 0] * ff[:, 2], ff[:, 0] * ff[:, 1]
    h = 1e-5
    fd = np.zeros(16)
    for c, comp in ((0, 0), (1, 1), (2, 2)):
        pp, pm = pts.copy(), pts.copy()
        pp[:, c] += h
        pm[:, c] -= h
        fd += (u_s(pp)[comp] - u_s(pm)[comp]) / (2 * h)
    np.testing.assert_allclose(e, fd, atol=1e-8)
    F, Fp = np.sin(3 * (pts[:, 1] - pts[:, 0])), 3 * np.cos(3 * (pts[:, 1] - pts[:, 0]))
    fw = np.stack([F, np.zeros(16), -F], 1)
    gw = np.zeros((16, 3, 3))
    gw[:, 0, 0], gw[:, 0, 1] = -Fp, Fp
    gw[:, 2, 0], gw[:, 2, 1] = Fp, -Fp
    assert np.abs(O.energy_residual(fw, gw, pts, W.MaxwellDesc())).max() < 1e-14


def test_ic_loss_closed_form():
    """At the IC plane the target is E_0 = exp(-25 (x^2 + y^2)), H = 0 (eqs. pulse_IC_*): the exact
    pulse gives L_IC = 0, and constant offsets (d, h1, h2) give d^2 + h1^2 + h2^2."""
    rng = np.random.default_rng(12)
    xy = rng.uniform(-1, 1, (32, 2))
    E0 = np.exp(-25 * (xy[:, 0] ** 2 + xy[:, 1] ** 2))
    desc = W.TotalLossDesc()
    z = np.zeros((4, 3)), np.zeros((4, 3, 3))
    pts = rng.uniform(-1, 1, (4, 3))
    f_ic = np.stack([E0, np.zeros(32), np.zeros(32)], 1)
    assert O.total_loss(z[0], z[1], z[0], z[0], f_ic, pts, xy, desc)["ic"] < 1e-30
    f_ic = np.stack([E0 + 0.1, np.full(32, 0.2), np.full(32, -0.3)], 1)
    assert O.total_loss(z[0], z[1], z[0], z[0], f_ic, pts, xy, desc)["ic"] == pytest.approx(0.14, rel=1e-12)


def test_symmetry_loss_parities():
    """Fields with the parities of eq. 2D_symLoss (E even in x and y, Hx even in x and odd in y,
    Hy odd in x and even in y) give L_sym = 0; adding c x to E breaks only the x-mirror parity:
    L_sym = mean((2 c x)^2) for the vacuum and 0 for the dielectric (x-mirror terms left out)."""
    rng = np.random.default_rng(13)
    pts = rng.uniform(-1, 1, (40, 3))

    def fields(p, c=0.0):
        t, x, y = p[:, 0], p[:, 1], p[:, 2]
        return np.stack([np.cos(2 * x) * np.cos(3 * y) * np.exp(-t) + c * x, np.cos(x) * np.sin(2 * y) * t,
                         np.sin(3 * x) * np.cos(y) + t * x], 1)
    mx, my = O.mirror_points(pts, 1), O.mirror_points(pts, 2)
    g = np.zeros((40, 3, 3))
    f_ic = np.zeros((0, 3))
    for kind in (W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT):
        d = W.TotalLossDesc(phys=W.MaxwellDesc(kind))
        assert O.total_loss(fields(pts), g, fields(mx), fields(my), f_ic, pts, np.zeros((0, 2)), d)["sym"] < 1e-28
    c = 0.3
    t = O.total_loss(fields(pts, c), g, fields(mx, c), fields(my, c), f_ic, pts, np.zeros((0, 2)), W.TotalLossDesc())
    assert t["sym"] == pytest.approx(np.mean((2 * c * pts[:, 1]) ** 2), rel=1e-12)
    d = W.TotalLossDesc(phys=W.MaxwellDesc(W.LOSS_DIEL_SPLIT))
    assert O.total_loss(fields(pts, c), g, fields(mx, c), fields(my, c), f_ic, pts, np.zeros((0, 2)), d)["sym"] < 1e-28


@pytest.mark.parametrize("kind", [W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT])
def test_total_loss_seeds_are_its_gradient(kind):
    rng = np.random.default_rng(14)
    P, P0 = 6, 5
    pts = rng.uniform(-1, 1, (P, 3))
    xy = rng.uniform(-1, 1, (P0, 2))
    arrs = [rng.standard_normal((P, 4)), rng.standard_normal((P, 4, 3)), rng.standard_normal((P, 4)),
            rng.standard_normal((P, 4)), rng.standard_normal((P0, 4))]
    desc = W.TotalLossDesc(phys=W.MaxwellDesc(kind, 4.0, 0.0), w_ic=3.0, w_sym=5.0, w_energy=7.0)
    seeds = O.total_loss_seeds(*arrs, pts, xy, desc)
    order = [0, 1, 2, 3, 4]
    seed_of = {0: seeds[0], 1: seeds[1], 2: seeds[2], 3: seeds[3], 4: seeds[4]}
    h = 1e-6
    for a in order:
        for idx in np.ndindex(*arrs[a].shape):
            pp = [x.copy() for x in arrs]
            pm = [x.copy() for x in arrs]
            pp[a][idx] += h
            pm[a][idx] -= h
            fd = (O.total_loss(*pp, pts, xy, desc)["total"] - O.total_loss(*pm, pts, xy, desc)["total"]) / (2 * h)
            assert fd == pytest.approx(seed_of[a][idx], abs=1e-7), (a, idx)


def test_total_loss_gradient_matches_fd():
    """Reverse mode over the four point sets with the total-loss seeds against central finite
    differences of L_tot in the parameters (forward simulations only)."""
    w = W.config(1, P=5)
    circ = W.layered(4, 2, "xyz", lambda l: W.ring(4, W.CNOT, 1))
    rng = np.random.default_rng(15)
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    xy = rng.uniform(-1, 1, (4, 2))
    for kind in (W.LOSS_VACUUM, W.LOSS_DIEL_SPLIT):
        desc = W.TotalLossDesc(phys=W.MaxwellDesc(kind, 4.0, 0.0))

        def L(prm):
            sets = [O.simulate(circ, prm, p)[0] for p in (O.mirror_points(w.points, 1), O.mirror_points(w.points, 2),
                                                          O.ic_points(xy))]
            f, g = O.simulate(circ, prm, w.points)
            return O.total_loss(f, g, sets[0], sets[1], sets[2], w.points, xy, desc)["total"]
        _, grad = O.total_eval(circ, params, w.points, xy, desc)
        h = 1e-6
        for k in (0, 5, 11, 17, 23):
            pp, pm = params.copy(), params.copy()
            pp[k] += h
            pm[k] -= h
            assert (L(pp) - L(pm)) / (2 * h) == pytest.approx(grad[k], rel=1e-8, abs=1e-8), (kind, k)


# ------------------------------------------------------------------------- diagnostics --------

def test_bloch_vectors_and_meyer_wallach_closed_forms():
    """Product state after RY(theta_q) embeddings and RX(a_q): r_q = (sin th cos.., ...) by the Bloch
    rotation; Meyer-Wallach 0 for every product state; GHZ (RY(pi/2) + CNOT chain) gives r = 0 on
    every qubit and Q = 1; a Bell pair plus an untouched qubit gives Q = 2/3."""
    n = 4
    rng = np.random.default_rng(21)
    th = rng.uniform(0, math.pi, (3, n))
    a = rng.uniform(0, 2 * math.pi, n)
    enc = W.Encoding(kind=W.ENC_ANGLES, gate=W.ENC_RY)
    circ = _circ(n, [(W.RX, q, -1, q) for q in range(n)], n, enc=enc, out=list(range(n)))
    r = O.bloch_vectors(circ, a, None, th, np.zeros((3, n, 3)))
    # RY(th)|0> has r = (sin th, 0, cos th); RX(a) rotates about x: (x, y cos a - z sin a, y sin a + z cos a)
    exp = np.stack([np.sin(th), -np.cos(th) * np.sin(a), np.cos(th) * np.cos(a)], -1)
    np.testing.assert_allclose(r, exp, atol=1e-12)
    np.testing.assert_allclose(O.meyer_wallach(circ, a, None, th, np.zeros((3, n, 3))), 0.0, atol=1e-12)
    ghz = _circ(n, [(W.RY, 0, -1, 0)] + [(W.CNOT, q, q + 1, -1) for q in range(n - 1)], 1, enc=enc,
                out=list(range(n)))
    z = np.zeros((1, n))
    np.testing.assert_allclose(O.bloch_vectors(ghz, [math.pi / 2], None, z, np.zeros((1, n, 3))), 0.0, atol=1e-12)
    assert O.meyer_wallach(ghz, [math.pi / 2], None, z, np.zeros((1, n, 3)))[0] == pytest.approx(1.0, abs=1e-12)
    bell = _circ(3, [(W.RY, 0, -1, 0), (W.CNOT, 0, 1, -1)], 1, enc=enc, out=[0, 1, 2])
    z3 = np.zeros((1, 3))
    assert O.meyer_wallach(bell, [math.pi / 2], None, z3, np.zeros((1, 3, 3)))[0] == pytest.approx(2 / 3, abs=1e-12)


def test_energy_profile_and_black_hole_indicator():
    """U(t) sums (eps E^2 + Hx^2 + Hy^2)/2 over the spatial grid per time slice: constant fields
    (1, 2, 3) on a 4 x 5 grid give 4 * 5 * (1 + 4 + 9) / 2 = 140 per slice (eps = 1); with eps = 4 on
    the points with x >= 0 those points count (4 + 4 + 9) / 2 each; I_BH of U = (2, 1.5, 0.2, 1) at
    t = (0, 0.05, 0.5, 1) with delta = 0.1 is 1 - 0.2 / 2 = 0.9."""
    t = np.array([0.0, 0.5, 1.0])
    xg, yg = np.linspace(-1, 1, 4), np.linspace(-1, 1, 5)
    pts = O.energy_grid(t, xg, yg)
    assert pts.shape == (60, 3) and np.all(pts[:20, 0] == 0.0) and np.all(pts[40:, 0] == 1.0)
    f = np.tile([1.0, 2.0, 3.0], (60, 1))
    np.testing.assert_allclose(O.energy_from_fields(f, pts, 3, W.MaxwellDesc()), 140.0)
    d = W.MaxwellDesc(W.LOSS_DIEL_SPLIT, 4.0, 0.0)
    n_diel = int(np.sum(xg >= 0)) * 5
    np.testing.assert_allclose(O.energy_from_fields(f, pts, 3, d), 0.5 * (n_diel * (4 + 13) + (20 - n_diel) * 14))
    assert O.black_hole_indicator([2.0, 1.5, 0.2, 1.0], [0.0, 0.05, 0.5, 1.0], 0.1) == pytest.approx(0.9)
