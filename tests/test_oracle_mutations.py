"""Planted mistakes in the CPU oracle must fail at least one of its pins (no GPU).

Each case swaps one oracle function for a copy carrying a plausible slip (a wrong sign, a dropped
factor or term, swapped operands or indices) and runs the fast pins of test_oracle_pins against
it.  A slip that no pin notices would mean the oracle is not pinned where the slip sits.
"""
import math

import numpy as np
import pytest

from oracle import qpinn_oracle as O
import workloads as W
import test_oracle_pins as pins

# the fast pins (each well under a second); the slow parameter-shift and 12-qubit cases are
# covered by the pin suite itself
FAST_PINS = [
    ("ry_embedding", pins.test_ry_embedding_closed_form, ()),
    ("rx_scaling_golden", pins.test_rx_scaling_identities_golden, ()),
    ("rx_embedding_phase", pins.test_rx_embedding_phase_closed_form, ()),
    ("scale_derivatives_fd", pins.test_scale_derivatives_match_finite_differences, ()),
    ("bloch_xyz", pins.test_product_state_matches_bloch_rotations, ("xyz", 3, 3)),
    ("bloch_rot", pins.test_product_state_matches_bloch_rotations, ("rot", 4, 2)),
    ("bell", pins.test_bell_state, ()),
    ("ghz_cnot_direction", pins.test_ghz_state_and_cnot_direction, ()),
    ("bitwise_sim_0", pins.test_kron_oracle_matches_bitwise_simulator, (0,)),
    ("bitwise_sim_1", pins.test_kron_oracle_matches_bitwise_simulator, (1,)),
    ("cz_sign_function", pins.test_cz_stride_ring_sign_function, ()),
    ("unitary_norm", pins.test_operators_unitary_and_norm_preserved, ()),
    ("init_zeros", pins.test_init_zeros_gives_unit_outputs, ()),
    ("trace_identity", pins.test_trace_identity_over_basis_encodings, ()),
    ("tangents_fd", pins.test_tangents_match_fd_and_encoding_shift, (1,)),
    ("rff_jacobian", pins.test_rff_jacobian_matches_fd, ()),
    ("param_shift_mixed", pins.test_reverse_mode_equals_parameter_shift, ("mixed",)),
    ("two_pi", pins.test_two_pi_periodicity, ()),
    ("plane_wave", pins.test_plane_wave_is_an_exact_zero_of_every_residual, ()),
    ("dielectric_weights", pins.test_dielectric_split_weights, ()),
    ("seeds_gradient", pins.test_seeds_are_the_gradient_of_the_loss_in_g, ()),
    ("bias_none_ry", pins.test_bias_and_none_scalings_closed_form_golden, (W.ENC_RY,)),
    ("bias_none_rx", pins.test_bias_and_none_scalings_closed_form_golden, (W.ENC_RX,)),
    ("rff_one_frequency", pins.test_rff_angles_one_frequency_closed_form, ()),
    ("crz_fd", pins.test_crz_gradient_matches_fd_of_loss, ()),
    ("crz_four_term_shift", pins.test_crz_gradient_matches_four_term_shift_rule, ()),
    ("input_grads_fd_ry", pins.test_input_gradients_match_fd, (W.ENC_RY,)),
    ("input_grads_shift_rx", pins.test_input_gradients_match_embedding_shift_rule, (W.ENC_RX,)),
    ("energy_poynting_vac", pins.test_energy_residual_is_the_poynting_balance, (W.LOSS_VACUUM,)),
    ("energy_poynting_diel", pins.test_energy_residual_is_the_poynting_balance, (W.LOSS_DIEL_SPLIT,)),
    ("ic_closed_form", pins.test_ic_loss_closed_form, ()),
    ("symmetry_parities", pins.test_symmetry_loss_parities, ()),
    ("total_seeds_vac", pins.test_total_loss_seeds_are_its_gradient, (W.LOSS_VACUUM,)),
]

_rotation = O.rotation
_full_operator = O.full_operator
_z_diagonal = O.z_diagonal
_readout = O.readout
_scale_derivative = O.scale_derivative
_embed_vectors = O._embed_vectors
_initial_states = O.initial_states
_maxwell_terms = O.maxwell_terms
_maxwell_seeds = O.maxwell_seeds
_grad_reverse = O.grad_reverse
_encoding_angles = O.encoding_angles
_scale_value = O.scale_value
_embed_second_derivative = O._embed_second_derivative
_energy_residual = O.energy_residual
_sym_terms = O._sym_terms
_ic_target = O.ic_target
_total_loss_seeds = O.total_loss_seeds


def rotation_sign(kind, theta):                       # exp(+i theta P / 2)
    return math.cos(theta / 2) * O.I2 + 1j * math.sin(theta / 2) * O.PAULI[kind]


def rotation_full_angle(kind, theta):                 # half angle dropped
    return math.cos(theta) * O.I2 - 1j * math.sin(theta) * O.PAULI[kind]


def rotation_derivative_no_half(kind, theta):         # -i P R instead of -(i/2) P R
    return -1j * O.PAULI[kind] @ _rotation(kind, theta)


def full_operator_cnot_swapped(n, kind, q0, q1, theta, derivative=False):
    if kind == O.CNOT:
        q0, q1 = q1, q0
    return _full_operator(n, kind, q0, q1, theta, derivative)


def full_operator_cz_as_cnot(n, kind, q0, q1, theta, derivative=False):
    return _full_operator(n, O.CNOT if kind == O.CZ else kind, q0, q1, theta, derivative)


def z_diagonal_reversed(n, i):                        # qubit order reversed in the readout
    return _z_diagonal(n, n - 1 - i)


def readout_without_two(circ, psi, dpsi):             # g = Re psi^H Z dpsi (factor 2 dropped)
    f, g = _readout(circ, psi, dpsi)
    return f, 0.5 * g


def scale_derivative_pi_dropped(kind, a):             # d(pi a)/da taken as 1
    if kind == O.SCALE_PI:
        return np.ones_like(a)
    return _scale_derivative(kind, a)


def embed_rx_conjugated(gate, theta):                 # RX(theta)|0> = (cos, +i sin)
    v, dv = _embed_vectors(gate, theta)
    if gate != O.ENC_RY:
        v, dv = np.conj(v), np.conj(dv)
    return v, dv


def initial_states_first_qubit_only(circ, theta, J):  # tangent terms of qubits >= 1 dropped
    J = np.array(J, copy=True)
    J[:, 1:, :] = 0.0
    return _initial_states(circ, theta, J)


def maxwell_terms_r3_sign(g, points, desc):           # r3 = dHy/dt + dE/dx
    r1, r2, r3, eps, w1, w = _maxwell_terms(g, points, desc)
    return r1, r2, g[:, 2, 0] + g[:, 0, 1], eps, w1, w


def maxwell_terms_weights_swapped(g, points, desc):   # 1/N_vac and 1/N_diel exchanged
    r1, r2, r3, eps, w1, w = _maxwell_terms(g, points, desc)
    if desc.kind == O.LOSS_DIEL_SPLIT:
        diel = np.asarray(points)[:, 1] >= desc.x_interface
        n_d = int(diel.sum())
        n_v = len(diel) - n_d
        w1 = np.where(diel, 1.0 / max(n_v, 1), 1.0 / max(n_d, 1))
    return r1, r2, r3, eps, w1, w


def maxwell_seeds_term_dropped(g, points, desc):      # dE/dy's share of r2 left out
    r1, r2, r3, eps, w1, w = _maxwell_terms(g, points, desc)
    W = _maxwell_seeds(g, points, desc)
    W[:, 0, 2] -= 2.0 * w * r2
    return W


def grad_reverse_sign(*a, **k):
    return -np.asarray(_grad_reverse(*a, **k))


def grad_reverse_tangent_seeds_dropped(circ, params, points, seeds_f, seeds_g, *a, **k):
    return _grad_reverse(circ, params, points, seeds_f, np.zeros_like(seeds_g), *a, **k)


def maxwell_terms_eps_multiplied(g, points, desc):    # eps multiplies the curl instead of dividing
    r1, r2, r3, eps, w1, w = _maxwell_terms(g, points, desc)
    curl = g[:, 2, 1] - g[:, 1, 2]
    return g[:, 0, 0] - curl * eps, r2, r3, eps, w1, w


def encoding_angles_rff_jacobian_sign(circ, *a, **k):
    theta, J = _encoding_angles(circ, *a, **k)
    if circ.enc.kind == O.ENC_RFF:
        J = -J
    return theta, J


def full_operator_crz_derivative_zero_branch(n, kind, q0, q1, theta, derivative=False):
    # d CRZ / d theta taken as P0 (x) I + P1 (x) dRZ (the constant branch not dropped)
    if kind == O.CRZ and derivative:
        return _full_operator(n, kind, q0, q1, theta, True) + _zero_branch(n, q0)
    return _full_operator(n, kind, q0, q1, theta, derivative)


def _zero_branch(n, q0):
    return O._kron_list([O.P0 if q == q0 else O.I2 for q in range(n)], n > O.DENSE_MAX_N)


def full_operator_crz_rx(n, kind, q0, q1, theta, derivative=False):
    # the controlled rotation taken about X instead of Z (forward and derivative alike)
    if kind != O.CRZ:
        return _full_operator(n, kind, q0, q1, theta, derivative)
    T = O.rotation_derivative(O.RX, theta) if derivative else O.rotation(O.RX, theta)
    one = O._kron_list([O.P1 if q == q0 else (T if q == q1 else O.I2) for q in range(n)], n > O.DENSE_MAX_N)
    return one if derivative else _zero_branch(n, q0) + one


def scale_value_bias_offset(kind, a):                 # (a - 1) pi/2: same derivative
    if kind == O.SCALE_BIAS:
        return (a - 1.0) * math.pi / 2.0
    return _scale_value(kind, a)


def scale_value_none_offset(kind, a):                 # a + pi/2: same derivative
    if kind == O.SCALE_NONE:
        return a + math.pi / 2.0
    return _scale_value(kind, a)


def _rff(circ, points, swap=False, two_pi=False):
    B = np.asarray(circ.enc.rff_B, np.float64)
    Wm = np.asarray(circ.enc.rff_W, np.float64)
    s = 2.0 * math.pi if two_pi else 1.0
    proj = s * (np.asarray(points, np.float64) @ B.T)
    a, b = np.cos(proj), np.sin(proj)
    da, db = -np.sin(proj), np.cos(proj)
    if swap:
        a, b, da, db = b, a, db, da
    phi = np.concatenate([a, b], axis=1)
    dphi = np.concatenate([da[:, :, None] * s * B[None], db[:, :, None] * s * B[None]], axis=1)
    return phi @ Wm.T, np.einsum("qf,pfc->pqc", Wm, dphi)


def encoding_angles_rff_cos_sin_swapped(circ, points, angles=None, jac=None):
    if circ.enc.kind == O.ENC_RFF:                    # [sin; cos] with a consistent Jacobian
        return _rff(circ, points, swap=True)
    return _encoding_angles(circ, points, angles, jac)


def encoding_angles_rff_two_pi(circ, points, angles=None, jac=None):
    if circ.enc.kind == O.ENC_RFF:                    # cos(2 pi B p) with a consistent Jacobian
        return _rff(circ, points, two_pi=True)
    return _encoding_angles(circ, points, angles, jac)


def embed_second_derivative_sign(gate, theta):      # +(1/4) v instead of -(1/4) v
    return -_embed_second_derivative(gate, theta)


def _input_grads_slipped(circ, theta, J, lam, mu, d_theta, d_J, cross=True, j_factor=2.0):
    P, n = theta.shape
    v, dv = O._embed_vectors(circ.enc.gate, theta)
    d2v = O._embed_second_derivative(circ.enc.gate, theta)
    for p in range(P):
        for q in range(n):
            t_q = O._kron_list([dv[p, qq] if qq == q else v[p, qq] for qq in range(n)], False)
            acc = np.vdot(lam[:, p], t_q)
            for c in range(3):
                d_J[p, q, c] = j_factor * np.real(np.vdot(mu[c, :, p], t_q))
                dd = J[p, q, c] * O._kron_list([d2v[p, qq] if qq == q else v[p, qq] for qq in range(n)], False)
                for q2 in range(n):
                    if cross and q2 != q:
                        dd = dd + J[p, q2, c] * O._kron_list(
                            [dv[p, qq] if qq in (q, q2) else v[p, qq] for qq in range(n)], False)
                acc += np.vdot(mu[c, :, p], dd)
            d_theta[p, q] = 2.0 * np.real(acc)


def input_grads_cross_terms_dropped(*a):            # d dpsi_c / d theta_q: only the q' = q term
    _input_grads_slipped(*a, cross=False)


def input_grads_jac_half(*a):                       # d/dJ = Re <mu, t_q> (factor 2 dropped)
    _input_grads_slipped(*a, j_factor=1.0)


def energy_residual_y_flux_sign(f, g, points, desc):   # + d(E Hx)/dy taken with a minus sign
    return _energy_residual(f, g, points, desc) - 2.0 * (g[:, 0, 2] * f[:, 1] + f[:, 0] * g[:, 1, 2])


def energy_residual_no_eps(f, g, points, desc):        # eps dropped from the electric energy
    eps = O._eps(points, desc)
    return _energy_residual(f, g, points, desc) - (eps - 1.0) * f[:, 0] * g[:, 0, 0]


def sym_terms_hx_even_in_y(f, f_mx, f_my, desc):       # (Hx - Hx^mirr_y)^2 instead of (Hx + ..)^2
    return _sym_terms(f, f_mx, f_my, desc) - (f[:, 1] + f_my[:, 1]) ** 2 + (f[:, 1] - f_my[:, 1]) ** 2


def ic_target_half_exponent(ic_xy, a):                 # exp(-a r^2 / 2)
    return _ic_target(ic_xy, a / 2.0)


def total_seeds_mirror_x_dropped(*a):                  # the x-mirror images get no seeds
    Vf, Wg, V_mx, V_my, V_ic = _total_loss_seeds(*a)
    return Vf, Wg, np.zeros_like(V_mx), V_my, V_ic


MUTATIONS = [
    ("rotation", rotation_sign),
    ("rotation", rotation_full_angle),
    ("rotation_derivative", rotation_derivative_no_half),
    ("full_operator", full_operator_cnot_swapped),
    ("full_operator", full_operator_cz_as_cnot),
    ("z_diagonal", z_diagonal_reversed),
    ("readout", readout_without_two),
    ("scale_derivative", scale_derivative_pi_dropped),
    ("_embed_vectors", embed_rx_conjugated),
    ("initial_states", initial_states_first_qubit_only),
    ("maxwell_terms", maxwell_terms_r3_sign),
    ("maxwell_terms", maxwell_terms_weights_swapped),
    ("maxwell_seeds", maxwell_seeds_term_dropped),
    ("grad_reverse", grad_reverse_sign),
    ("grad_reverse", grad_reverse_tangent_seeds_dropped),
    ("maxwell_terms", maxwell_terms_eps_multiplied),
    ("encoding_angles", encoding_angles_rff_jacobian_sign),
    ("full_operator", full_operator_crz_derivative_zero_branch),
    ("full_operator", full_operator_crz_rx),
    ("scale_value", scale_value_bias_offset),
    ("scale_value", scale_value_none_offset),
    ("encoding_angles", encoding_angles_rff_cos_sin_swapped),
    ("encoding_angles", encoding_angles_rff_two_pi),
    ("_embed_second_derivative", embed_second_derivative_sign),
    ("_input_grads", input_grads_cross_terms_dropped),
    ("_input_grads", input_grads_jac_half),
    ("energy_residual", energy_residual_y_flux_sign),
    ("energy_residual", energy_residual_no_eps),
    ("_sym_terms", sym_terms_hx_even_in_y),
    ("ic_target", ic_target_half_exponent),
    ("total_loss_seeds", total_seeds_mirror_x_dropped),
]


def _caught(monkeypatch, name, fn):
    caught = []
    with monkeypatch.context() as m:
        m.setattr(O, name, fn)
        for label, pin, args in FAST_PINS:
            try:
                pin(*args)
            except Exception:
                caught.append(label)
    return caught


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[f.__name__ for _, f in MUTATIONS])
def test_planted_mistake_fails_a_pin(monkeypatch, name, fn):
    caught = _caught(monkeypatch, name, fn)
    assert caught, f"no pin notices {fn.__name__} in oracle.{name}"


def test_unmutated_oracle_passes_the_fast_pins(monkeypatch):
    assert _caught(monkeypatch, "rotation", _rotation) == []
