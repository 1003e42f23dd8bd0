"""Full-size workloads in the launch configuration bench.py times (GPU only).

The oracle cannot evaluate hundreds of thousands of 12-qubit gradients, so at full size the
outputs and tangents are compared with the oracle on sampled points (spread over the point
range, both ends included), and the loss and gradient through properties that hold at any size:
with the summed loss (QP_FLAG_LOSS_SUM) both are additive over a partition of the points, and a
repeated call is bitwise identical.
"""
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


@pytest.mark.parametrize("k", [4, 2])
def test_full_size_sampled_outputs_and_additive_gradient(ctx, k):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    w = W.config(k)
    P = len(w.points)
    c = Circuit(ctx, w.circuit)
    r = c.maxwell(w.params, w.points, w.loss)
    out, tan = t2n(r["out"]).copy(), t2n(r["tan"]).copy()
    grad_mean = t2n(r["grad"]).copy()
    # sampled outputs and tangents against the oracle
    idx = np.unique(np.r_[np.linspace(0, P - 1, 10).astype(int), [1, P - 2]])
    f, g = O.simulate(w.circuit, w.params, w.points[idx])
    e_f, e_g = rel(out[idx], f), rel(tan[idx], g)
    report(f"full size {w.name} P={P} sampled {len(idx)}", f=e_f, g=e_g)
    assert e_f < TOL and e_g < TOL
    # repeat: bitwise identical
    r2 = c.maxwell(w.params, w.points, w.loss)
    assert np.array_equal(t2n(r2["grad"]), grad_mean)
    assert np.array_equal(t2n(r2["out"]), out)
    assert np.all(np.isfinite(grad_mean))
    # summed loss is additive over a partition of the points (ragged split inside a tile)
    if w.loss.kind == W.LOSS_VACUUM:
        cut = P // 3 + 1
        full = c.maxwell(w.params, w.points, w.loss, flags=L.QP_FLAG_LOSS_SUM)
        lf, gf = float(t2n(full["loss"])[0]), t2n(full["grad"]).copy()
        a = c.maxwell(w.params, w.points[:cut], w.loss, flags=L.QP_FLAG_LOSS_SUM)
        la, ga = float(t2n(a["loss"])[0]), t2n(a["grad"]).copy()
        b = c.maxwell(w.params, w.points[cut:], w.loss, flags=L.QP_FLAG_LOSS_SUM)
        lb, gb = float(t2n(b["loss"])[0]), t2n(b["grad"]).copy()
        e_l, e_gr = abs(lf - (la + lb)) / abs(lf), rel(gf, ga + gb)
        report(f"full size {w.name} additivity", loss=e_l, grad=e_gr)
        assert e_l < TOL and e_gr < TOL
        # and the mean loss is the summed loss over P
        assert abs(float(t2n(r["loss"])[0]) - lf / P) <= TOL * abs(lf / P)
        assert rel(grad_mean, gf / P) < TOL


def test_eight_times_the_full_size(ctx):
    """The 12-qubit circuit on 2^21 + 37 points (eight times the full-size workload, fresh seeded
    draw): sampled outputs and tangents against the oracle, and the summed loss and gradient
    additive over a split of the points."""
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    w = W.config(4)
    P = (1 << 21) + 37
    pts = W.uniform_points(np.random.default_rng(2106), P, np.float32)
    c = Circuit(ctx, w.circuit)
    full = c.maxwell(w.params, pts, w.loss, flags=L.QP_FLAG_LOSS_SUM)
    out, tan = t2n(full["out"]), t2n(full["tan"])
    idx = np.unique(np.r_[np.linspace(0, P - 1, 8).astype(int), [P - 2]])
    f, g = O.simulate(w.circuit, w.params, pts[idx])
    e_f, e_g = rel(out[idx], f), rel(tan[idx], g)
    report(f"{w.name} P={P} sampled {len(idx)}", f=e_f, g=e_g)
    assert e_f < TOL and e_g < TOL
    lf, gf = float(t2n(full["loss"])[0]), t2n(full["grad"]).copy()
    cut = (1 << 20) + 1
    a = c.maxwell(w.params, pts[:cut], w.loss, flags=L.QP_FLAG_LOSS_SUM, outputs=False)
    b = c.maxwell(w.params, pts[cut:], w.loss, flags=L.QP_FLAG_LOSS_SUM, outputs=False)
    la, lb = float(t2n(a["loss"])[0]), float(t2n(b["loss"])[0])
    e_l, e_gr = abs(lf - (la + lb)) / abs(lf), rel(gf, t2n(a["grad"]) + t2n(b["grad"]))
    report(f"{w.name} P={P} additivity", loss=e_l, grad=e_gr)
    assert np.isfinite(lf) and np.all(np.isfinite(gf))
    assert e_l < TOL and e_gr < TOL
