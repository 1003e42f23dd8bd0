"""Dense 2^5-block path on FP32 MFMA (QP_FLAG_DENSE_MFMA) vs the oracle (GPU only)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.gpu_helpers import TOL, rel, report, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_23246_amd.api import Context
    return Context(0)


def _flags():
    from paper_2506_23246_amd import _lib as L
    return L.QP_FLAG_DENSE_MFMA


def _circ(ctx, c):
    from paper_2506_23246_amd.api import Circuit
    return Circuit(ctx, c)


@pytest.mark.parametrize("k,P", [(1, 100), (2, 70), (4, 64)])
def test_dense_forward_configs(ctx, k, P):
    w = W.config(k, P=P)
    c = _circ(ctx, w.circuit)
    out, tan = c.simulate(w.params, w.points, flags=_flags())
    f, g = O.simulate(w.circuit, w.params, w.points)
    e = dict(f=rel(t2n(out), f), g=rel(t2n(tan), g))
    report(f"dense forward {w.name} P={P}", **e)
    assert e["f"] < TOL and e["g"] < TOL


@pytest.mark.parametrize("k,P", [(1, 100), (2, 70), (4, 64)])
def test_dense_maxwell_configs(ctx, k, P):
    w = W.config(k, P=P)
    c = _circ(ctx, w.circuit)
    r = c.maxwell(w.params, w.points, w.loss, flags=_flags())
    f, g, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    e = dict(f=rel(t2n(r["out"]), f), g=rel(t2n(r["tan"]), g), loss=rel(t2n(r["loss"]), [L]),
             grad=rel(t2n(r["grad"]), grad))
    report(f"dense maxwell {w.name} P={P}", **e)
    for key, v in e.items():
        assert v < TOL, (key, v)


def test_dense_vjp_mixed_rings(ctx):
    rng = np.random.default_rng(31)
    n = 7
    rings = [W.ring(n, W.CNOT, 1) + W.ring(n, W.CZ, 2), W.ring(n, W.CZ, 1), W.ring(n, W.CNOT, 3)]
    circ = W.layered(n, 3, "xyz", lambda l: rings[l], out_qubits=[0, 6, 3])
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    pts = rng.uniform(-1, 1, (40, 3)).astype(np.float32)
    d_out = rng.standard_normal((40, 3)).astype(np.float32)
    d_tan = rng.standard_normal((40, 3, 3)).astype(np.float32)
    c = _circ(ctx, circ)
    got = t2n(c.vjp(params, pts, d_out, d_tan, flags=_flags()))
    exp = O.grad_reverse(circ, params, pts, d_out, d_tan)
    e = rel(got, exp)
    report("dense vjp mixed rings", grad=e)
    assert e < TOL


def test_dense_cross_mesh_crz(ctx):
    """The paper's Cross-Mesh ansatz (RX + all-pairs CRZ, eq. crz_cross_mesh) at 7 qubits, 2 layers,
    with per-point angles: only the dense path runs parametrised two-qubit gates."""
    rng = np.random.default_rng(32)
    circ = W.cross_mesh(7, 2, "x", W.CRZ, enc=W.Encoding(kind=W.ENC_ANGLES, gate=W.ENC_RX))
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 30
    ang = rng.uniform(0, math.pi, (P, 7)).astype(np.float32)
    jac = rng.standard_normal((P, 7, 3)).astype(np.float32)
    c = _circ(ctx, circ)
    out, tan = c.simulate(params, None, ang, jac, flags=_flags())
    f, g = O.simulate(circ, params, None, ang, jac)
    d_tan = rng.standard_normal((P, 3, 3)).astype(np.float32)
    got = t2n(c.vjp(params, None, None, d_tan, ang, jac, flags=_flags()))
    exp = O.grad_reverse(circ, params, None, None, d_tan, ang, jac)
    e = dict(f=rel(t2n(out), f), g=rel(t2n(tan), g), grad=rel(got, exp))
    report("dense cross-mesh CRZ", **e)
    for key, v in e.items():
        assert v < TOL, (key, v)


def test_dense_matches_fused_on_c5_chunked(ctx):
    """12 qubits on 20000 points (more than one dense chunk): dense and fused agree."""
    w = W.config(4, P=20000)
    c = _circ(ctx, w.circuit)
    rd = c.maxwell(w.params, w.points, w.loss, flags=_flags())
    rd = {k: t2n(v).copy() for k, v in rd.items()}
    rf = {k: t2n(v).copy() for k, v in c.maxwell(w.params, w.points, w.loss).items()}
    e = {k: rel(rd[k], rf[k]) for k in rd}
    report("dense vs fused c5 P=20000", **e)
    for key, v in e.items():
        assert v < 2 * TOL, (key, v)


@pytest.mark.parametrize("name,chunk", [("c5_first4096", 1024), ("c5_first4096", 0), ("c3_first16384", 4096)])
def test_dense_multi_chunk_against_stored_oracle(ctx, name, chunk):
    """Several point chunks through HBM (chunk 1024 or 4096: four chunks) and the default chunk:
    outputs, tangents, loss and gradient against the stored oracle results of the whole set."""
    from tests.golden.make_oracle_fixtures import SETS, load
    w = SETS[name]()
    ref = load(name)
    c = _circ(ctx, w.circuit)
    c.set_dense_chunk(chunk)
    r = c.maxwell(w.params, w.points, w.loss, flags=_flags())
    idx = ref["idx"]
    e = dict(f=rel(t2n(r["out"])[idx], ref["f"]), g=rel(t2n(r["tan"])[idx], ref["g"]),
             loss=rel(t2n(r["loss"]), [float(ref["loss"])]), grad=rel(t2n(r["grad"]), ref["grad"]))
    report(f"dense stored oracle {name} chunk {chunk}", **e)
    for key, v in e.items():
        assert v < TOL, (key, v)


@pytest.mark.parametrize("n,out", [(5, [4, 0, 2, 1, 3]), (9, [8, 1, 7, 2, 6, 3, 5, 0])])
def test_dense_readout_slices_and_output_counts(ctx, n, out):
    """The readout's amplitude slices at their extremes: 5 qubits (one 32-amplitude slice, three
    idle waves of the slice group) and 9 qubits (16 slices in 4 groups) with 8 read-out qubits in
    scrambled order; forward, tangents and the VJP against the oracle."""
    rng = np.random.default_rng(40 + n)
    circ = W.layered(n, 2, "xyz", lambda l: W.ring(n, W.CNOT if l == 0 else W.CZ, 1), out_qubits=out)
    params = rng.uniform(0, 2 * math.pi, circ.n_params).astype(np.float32)
    P = 70
    pts = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    m = len(out)
    d_out = rng.standard_normal((P, m)).astype(np.float32)
    d_tan = rng.standard_normal((P, m, 3)).astype(np.float32)
    c = _circ(ctx, circ)
    f_got, g_got = c.simulate(params, pts, flags=_flags())
    f, g = O.simulate(circ, params, pts)
    got = t2n(c.vjp(params, pts, d_out, d_tan, flags=_flags()))
    exp = O.grad_reverse(circ, params, pts, d_out, d_tan)
    e = dict(f=rel(t2n(f_got), f), g=rel(t2n(g_got), g), grad=rel(got, exp))
    report(f"dense readout {n}q, {m} outputs", **e)
    for key, v in e.items():
        assert v < TOL, (key, v)
