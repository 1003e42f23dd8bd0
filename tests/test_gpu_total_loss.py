"""The paper's total loss (eq. 2D_lossTot: residuals + 10 IC + 10 symmetry + 10 energy) on the GPU
against the CPU oracle: the four terms, their weighted sum and the parameter gradient, normwise
relative error per quantity, bar 1e-5.  At the full 12-qubit size the terms are checked against
the oracle's loss function applied to the library's own outputs and tangents (a property that
holds at any size; the outputs themselves are pinned by the other parity tests)."""
import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.gpu_helpers import TOL, rel, report, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_23246_amd.api import Context
    assert torch.cuda.is_available()
    return Context(0)


def _ic(n, seed):
    return W.ic_plane_points(np.random.default_rng(seed), n)


@pytest.mark.parametrize("k,P,P0", [(1, 40, 30), (2, 24, 16), (4, 3, 2), (1, 0, 12), (1, 17, 0)])
def test_total_loss_matches_oracle(ctx, k, P, P0):
    from paper_2506_23246_amd.api import Circuit
    w = W.config(k, P=max(P, 1))
    pts = w.points[:P]
    xy = _ic(P0, 40 + k)
    desc = W.TotalLossDesc(phys=w.loss)
    c = Circuit(ctx, w.circuit)
    r = c.total_loss(w.params, pts, xy, desc, outputs=True)
    terms, grad = O.total_eval(w.circuit, w.params, pts, xy, desc)
    got = t2n(r["terms"])
    ref = np.array([terms["total"], terms["phys"], terms["ic"], terms["sym"], terms["energy"]])
    errs = {name: rel([got[i]], [ref[i]]) if ref[i] != 0 else abs(got[i])
            for i, name in enumerate(["total", "phys", "ic", "sym", "energy"])}
    errs["grad"] = rel(t2n(r["grad"]), grad)
    if P:
        f, g = O.simulate(w.circuit, w.params, pts)
        errs["f"], errs["g"] = rel(t2n(r["out"]), f), rel(t2n(r["tan"]), g)
    report(f"total loss config {k} P={P} P0={P0}", **errs)
    assert all(v < TOL for v in errs.values()), errs


def test_total_loss_parameter_free_circuit(ctx):
    """A circuit with no trainable gate (K = 0, entangler rings only): the collocation pass forms
    no gradient; the four terms, outputs and tangents against the oracle."""
    from paper_2506_23246_amd.api import Circuit
    circ = W.Circuit(n=5, gates=W.ring(5, W.CNOT, 1) + W.ring(5, W.CZ, 2), n_params=0)
    params = np.zeros(0, np.float32)
    rng = np.random.default_rng(77)
    pts = rng.uniform(-1, 1, (70, 3)).astype(np.float32)
    xy = _ic(20, 78)
    desc = W.TotalLossDesc(phys=W.MaxwellDesc(W.LOSS_VACUUM))
    c = Circuit(ctx, circ)
    r = c.total_loss(params, pts, xy, desc, outputs=True)
    terms, _ = O.total_eval(circ, params, pts, xy, desc)
    got = t2n(r["terms"])
    ref = np.array([terms["total"], terms["phys"], terms["ic"], terms["sym"], terms["energy"]])
    errs = {name: rel([got[i]], [ref[i]]) if ref[i] != 0 else abs(got[i])
            for i, name in enumerate(["total", "phys", "ic", "sym", "energy"])}
    f, g = O.simulate(circ, params, pts)
    errs["f"], errs["g"] = rel(t2n(r["out"]), f), rel(t2n(r["tan"]), g)
    report("total loss K=0", **errs)
    assert all(v < TOL for v in errs.values()), errs


def test_total_loss_full_size_terms_follow_from_outputs(ctx):
    """12 qubits x 8 layers at 262144 collocation points and a 4096-point IC plane: the four terms
    equal the oracle's loss function applied to the library's outputs and tangents of the four
    point sets (taken with qp_simulate), and a repeated call is bitwise identical."""
    import torch
    from paper_2506_23246_amd.api import Circuit
    w = W.config(4)
    xy = _ic(4096, 7)
    desc = W.TotalLossDesc(phys=w.loss)
    c = Circuit(ctx, w.circuit)
    r = c.total_loss(w.params, w.points, xy, desc)
    got = t2n(r["terms"]).copy()
    g1 = t2n(r["grad"]).copy()
    sets = {}
    for name, pts in (("x", w.points), ("mx", O.mirror_points(w.points, 1)), ("my", O.mirror_points(w.points, 2)),
                      ("ic", O.ic_points(xy))):
        out, tan = c.simulate(w.params, pts.astype(np.float32))
        sets[name] = (t2n(out), t2n(tan))
    terms = O.total_loss(sets["x"][0], sets["x"][1], sets["mx"][0], sets["my"][0], sets["ic"][0], w.points, xy, desc)
    ref = np.array([terms["total"], terms["phys"], terms["ic"], terms["sym"], terms["energy"]])
    errs = {name: rel([got[i]], [ref[i]]) for i, name in enumerate(["total", "phys", "ic", "sym", "energy"])}
    report("total loss full size", **errs)
    assert all(v < TOL for v in errs.values()), errs
    r2 = c.total_loss(w.params, w.points, xy, desc)
    assert np.array_equal(t2n(r2["grad"]), g1) and np.array_equal(t2n(r2["terms"]), got)
    assert np.all(np.isfinite(g1))
    torch.cuda.synchronize()


def test_total_loss_rejects_the_angle_encoding(ctx):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    circ = W.paper_context_circuit("basic")
    c = Circuit(ctx, circ)
    with pytest.raises(L.QPError) as e:
        c.total_loss(np.zeros(circ.n_params, np.float32), np.zeros((4, 3), np.float32), _ic(2, 1),
                     W.TotalLossDesc())
    assert e.value.status == L.QP_EINVAL
