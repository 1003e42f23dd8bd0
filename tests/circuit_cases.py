"""Circuits that open in different ways, for the planner's fold of an opening rotation stage into
the product-state encoding (shared by the CPU emulation tests and the GPU parity tests)."""
import workloads as W


def _circ(n, gates, n_params, out_qubits=(0, 1, 2)):
    return W.Circuit(n=n, gates=list(gates), n_params=n_params, out_qubits=list(out_qubits))


def opening_stage_cases():
    """Circuits that open in different ways: (name, circuit, expected number of folded rounds)."""
    cases = []
    n = 6   # no swap slots: 3 gates per round
    g = W.ring(n, W.CNOT, 1)
    c = W.layered(n, 2, "xyz", lambda l: W.ring(n, W.CNOT, 1))
    cases.append(("rotations first", c, 2))
    c = _circ(n, g + W.layered(n, 2, "xz", lambda l: W.ring(n, W.CZ, 1)).gates, 4 * n)
    cases.append(("entangler first", c, 0))
    # leading stage on qubits 1 and 4 only, then a ring, then a full layer
    gates = [(W.RY, 1, -1, 0), (W.RZ, 4, -1, 1)] + g + W.layered(n, 1, "xyz").gates
    gates = [(k, q0, q1, (p + 2) if (p >= 0 and i >= 2 + len(g)) else p) for i, (k, q0, q1, p) in enumerate(gates)]
    cases.append(("partial leading stage", _circ(n, gates, 2 + 3 * n), 1))
    # four rotations on qubit 0 split the opening rotations into two stages; only the first folds
    gates = [(W.RX, 0, -1, 0), (W.RY, 0, -1, 1), (W.RZ, 0, -1, 2), (W.RY, 0, -1, 3), (W.RX, 2, -1, 4)] + g + \
        [(W.RY, q, -1, 5 + q) for q in range(n)]
    cases.append(("split opening rotations", _circ(n, gates, 5 + n), 1))
    # no entangler at all: every round but the last folds
    cases.append(("no entangler", W.layered(n, 1, "xyz"), 1))
    # 10 qubits (two swap slots, 5 gates a round) and 8 qubits (one swap slot) with a CZ ring
    cases.append(("10 qubits", W.layered(10, 2, "rot", lambda l: W.ring(10, W.CZ, 2)), 2))
    cases.append(("8 qubits", W.layered(8, 2, "xyz", lambda l: W.ring(8, W.CNOT, 3), out_qubits=[0, 7, 3]), 2))
    return cases
