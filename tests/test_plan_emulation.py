"""Host logic: the planner's device image, executed by a CPU emulation of the fused kernel's
register/LDS algorithm, reproduces the oracle (outputs, tangents and parameter gradients)."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.circuit_cases import opening_stage_cases

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2506_23246_amd",
                   "libqpinn.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _run(circ, params, pts, seeds=True):
    from tests.plan_emulator import emulate_point, grads_from_m, grads_from_s, plan_image
    plan = plan_image(circ)
    theta, J = O.encoding_angles(circ, pts)
    f, g = O.simulate(circ, params, pts)
    Wg = O.maxwell_seeds(g, pts, W.MaxwellDesc()) if seeds else None
    M = S = 0
    for p in range(len(pts)):
        fe, ge, Mp, Sp = emulate_point(plan, params, theta[p], J[p], circ.enc.gate == W.ENC_RX,
                                   None, Wg[p] if seeds else None)
        np.testing.assert_allclose(fe, f[p], atol=1e-12)
        np.testing.assert_allclose(ge, g[p], atol=1e-11)
        if seeds:
            M = M + Mp
            S = S + Sp
    if seeds:
        exp = O.grad_reverse(circ, params, pts, None, Wg)
        np.testing.assert_allclose(grads_from_m(plan, params, M), exp, atol=1e-11)
        # the kernel's statistic: Pauli components with the rotated generator axes
        np.testing.assert_allclose(grads_from_s(plan, params, S), exp, atol=1e-11)
        # ... also when every gate's statistic is taken at its round's input (pipelined kernel)
        S2 = 0
        for p in range(len(pts)):
            S2 = S2 + emulate_point(plan, params, theta[p], J[p], circ.enc.gate == W.ENC_RX, None, Wg[p],
                                    stats_at_round_input=True)[3]
        np.testing.assert_allclose(grads_from_s(plan, params, S2), exp, atol=1e-11)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_emulated_plan_matches_oracle_on_configs(k):
    w = W.config(k, P=3)
    if k == 0:
        w.circuit.out_qubits = [0, 1, 2]
    _run(w.circuit, np.asarray(w.params, np.float64), np.asarray(w.points, np.float64))


@pytest.mark.parametrize("n", [3, 4, 5, 7, 9, 10, 12])
def test_emulated_plan_mixed_entanglers(n):
    """Mixed CNOT/CZ rings of several strides; 10 qubits exercise two swap slots per round."""
    rng = np.random.default_rng(n)
    rings = [W.ring(n, W.CNOT, 1) + W.ring(n, W.CZ, 2), W.ring(n, W.CZ, 1), W.ring(n, W.CNOT, 2)]
    layers = 3 if n <= 10 else 2
    circ = W.layered(n, layers, "xyz", lambda l: rings[l], out_qubits=[0, n - 1, n // 2])
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    pts = rng.uniform(-1, 1, (2 if n <= 10 else 1, 3))
    _run(circ, params, pts)


@pytest.mark.parametrize("case", range(7))
def test_leading_stage_folding(case):
    """The planner folds exactly the rounds of an opening rotation stage (one gate per qubit, acting
    on the product state), except the circuit's last round, into the encoding; those gates take
    their statistic at the gate output.
    The emulated kernel, which forms the product state with those gates applied and takes their
    statistics without pulling anything back, matches the oracle's outputs, tangents and gradient."""
    from tests.plan_emulator import plan_image
    name, circ, nh = opening_stage_cases()[case]
    plan = plan_image(circ)
    h = plan["h"]
    assert int(h["n_head"]) == nh, name
    head = {int(h["head_gate"][q]) for q in range(circ.n) if int(h["head_gate"][q]) >= 0}
    in_rounds = set()
    for k in range(nh):
        rd = plan["rounds"][k]
        in_rounds |= {int(x) for x in list(rd["gate"]) + list(rd["sgate"]) if int(x) >= 0}
    assert head == in_rounds, name
    for fi, f in enumerate(plan["fused"]):
        assert int(f["stat_out"]) == (1 if fi in head else 0), name
        if fi in head:
            assert int(h["head_gate"][int(f["qubit"])]) == fi
    rng = np.random.default_rng(100 + case)
    params = rng.uniform(0, 2 * math.pi, circ.n_params)
    pts = rng.uniform(-1, 1, (2, 3))
    _run(circ, params, pts)


def test_leading_stage_of_the_twelve_qubit_workload():
    """12 qubits x 8 layers: three rounds of four gates per layer (one swap slot), and the first
    layer's twelve gates are the three folded rounds."""
    from tests.plan_emulator import plan_image
    plan = plan_image(W.config(4, P=1).circuit)
    h = plan["h"]
    assert int(h["n_rounds"]) == 24 and int(h["n_head"]) == 3
    assert sorted(int(x) for x in h["head_gate"][:12]) == list(range(12))
    assert all(int(x) == -1 for x in h["head_gate"][12:])


def _lane_cases():
    rng_rings = lambda n: [W.ring(n, W.CNOT, 1) + W.ring(n, W.CZ, 2), W.ring(n, W.CZ, 1), W.ring(n, W.CNOT, 2)]
    out = [W.config(k, P=1).circuit for k in (1, 2, 4)]
    for n in (3, 5, 8, 10, 11):
        rings = rng_rings(n)
        out.append(W.layered(n, 3, "xyz", lambda l, rings=rings: rings[l], out_qubits=[0, n - 1, n // 2]))
    return out


@pytest.mark.parametrize("case", range(8))
def test_plan_lane_words(case):
    """The planner's per-lane exchange words (writer base, reader base, sign bits per register),
    which the kernel loads instead of deriving them, agree for every exchange and thread with the
    writer's deposit and with the reader side computed from the exchange descriptor alone (GF(2)
    index-map columns and the bilinear split of the CZ sign form), an independent derivation; both
    bases through the exchange's LDS layout map M."""
    from tests.plan_emulator import _deposit, _swz, descriptor_words, plan_image
    circ = _lane_cases()[case]
    plan = plan_image(circ)
    n, R = circ.n, int(plan["h"]["n_rounds"])
    TP = 1 << (n - 3)
    rounds, L = plan["rounds"], plan["lanes"]
    assert L.shape == (2, R, TP)
    for k in range(1, R):
        for d, (wmap, rmap, X) in enumerate([(rounds[k - 1]["tpost"], rounds[k]["tpos"], plan["xf"][k]),
                                             (rounds[k]["tpos"], rounds[k - 1]["tpost"], plan["xb"][k])]):
            M = [int(c) for c in X["mcol"][:n]]
            for u in range(TP):
                lw = L[d, k, u]
                assert int(lw["wb"]) == 8 * _swz(_apply_cols(M, _deposit(u, wmap, n))), (case, k, d, u)
                sb, _, sg = descriptor_words(X, n, rmap, u)
                assert int(lw["rb"]) == 8 * _swz(_apply_cols(M, sb)), (case, k, d, u)
                assert int(lw["sgn"]) == sum(b << r for r, b in enumerate(sg)), (case, k, d, u)
    for f in ("wb", "rb", "sgn"):   # round 0 has no exchange
        assert np.all(L[:, 0][f] == 0)


def _swz(i):
    return i ^ (((i >> 4) ^ (i >> 8) ^ (i >> 12) ^ (i >> 16)) & 15)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_plan_lds_offset_tables(k):
    """The planner's LDS layout per exchange: logical index j at entry swz(pbase ^ M j) with M
    invertible over GF(2); writer offsets woff[r] = 8 swz(M jr(r)) in the writer's mapping and
    reader offsets roff[r] = 8 swz(M A jr(r)) in the reader's mapping (forward exchanges read into
    a round's input mapping, reverse ones into the previous round's output mapping).  swz must be
    linear over GF(2), which the kernel's address arithmetic relies on, and the layout must give
    every group of 16 lanes distinct banks (low four entry bits) on both sides of every exchange at
    8 and 12 qubits, which is what M is chosen for, and never fewer than the plain swizzle."""
    from tests.plan_emulator import _deposit, _regoff, plan_image
    circ = W.config(k, P=1).circuit
    plan = plan_image(circ)
    n = circ.n
    rounds = plan["rounds"]
    R = len(rounds)
    T = 512 if n == 12 else 256
    TP = 1 << (n - 3)
    distinct, plain = [], []
    for kk in range(1, R):
        for X, wmap, rmap in ((plan["xf"][kk], rounds[kk - 1]["tpost"], rounds[kk]["tpos"]),
                              (plan["xb"][kk], rounds[kk]["tpos"], rounds[kk - 1]["tpost"])):
            M = [int(c) for c in X["mcol"][:n]]
            A = [int(c) for c in X["acol"][:n]]
            assert _gf2_rank(M) == n
            for r in range(8):
                assert int(X["woff"][r]) == 8 * _swz(_apply_cols(M, _regoff(r, wmap)))
                assert int(X["roff"][r]) == 8 * _swz(_apply_cols(M, _apply_cols(A, _regoff(r, rmap))))
            for side in range(2):
                for h0 in range(0, T, 16):
                    banks, banks0 = set(), set()
                    for t in range(h0, h0 + 16):
                        ps, u = divmod(t, TP)
                        j = _deposit(u, wmap, n) if side == 0 else _apply_cols(A, _deposit(u, rmap, n))
                        banks.add(_swz((ps << n) ^ _apply_cols(M, j)) & 15)
                        banks0.add(_swz((ps << n) ^ j) & 15)
                    distinct.append(len(banks))
                    plain.append(len(banks0))
    assert np.mean(distinct) >= np.mean(plain)
    if n >= 8:
        assert np.mean(distinct) == 16.0, np.mean(distinct)
    rng = np.random.default_rng(0)
    for a, b in rng.integers(0, 1 << 12, (200, 2)):
        assert _swz(int(a) ^ int(b)) == _swz(int(a)) ^ _swz(int(b))


def _apply_cols(cols, x):
    y, k = 0, 0
    while x:
        if x & 1:
            y ^= cols[k]
        x >>= 1
        k += 1
    return y


def _gf2_rank(cols):
    rows, r = list(cols), 0
    for bit in range(32):
        piv = next((i for i in range(r, len(rows)) if (rows[i] >> bit) & 1), None)
        if piv is None:
            continue
        rows[r], rows[piv] = rows[piv], rows[r]
        for i in range(len(rows)):
            if i != r and (rows[i] >> bit) & 1:
                rows[i] ^= rows[r]
        r += 1
    return r


@pytest.mark.parametrize("n", [8, 9, 10, 11, 12])
def test_plan_swap_slots(n):
    """Rounds of a full rotation stage fill the register bits and the swap slots: n = 8, 9, 10, 11, 12
    need 2, 3, 2, 4, 3 rounds per layer (one swap slot at 8 and 12 qubits, two at 10); the output mapping
    is the input mapping with register bit i and thread bit 4 + i exchanged for every swap slot."""
    from tests.plan_emulator import _swap_slots, plan_image
    circ = W.layered(n, 2, "xyz", lambda l: W.ring(n, W.CNOT, 1), out_qubits=[0, 1, 2])
    plan = plan_image(circ)
    rounds = plan["rounds"]
    per_layer = {8: 2, 9: 3, 10: 2, 11: 4, 12: 3}[n]
    assert len(rounds) == 2 * per_layer
    nsw = _swap_slots(n)
    for rd in rounds:
        t, tp = list(rd["tpos"][:n]), list(rd["tpost"][:n])
        assert sorted(t) == list(range(n))
        for i in range(nsw):
            t[i], t[7 + i] = t[7 + i], t[i]
        assert t == tp
