"""Uneven batch (many circuits, one persistent launch) vs the oracle, vs the single-circuit
fused path, and under hipGraph replay (GPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import qpinn_oracle as O
from tests.gpu_helpers import TOL, rel, report, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_23246_amd.api import Context
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    return Context(0, stream=s), s


def _batch(ctx, ws):
    from paper_2506_23246_amd.api import Batch
    return Batch(ctx, [w.circuit for w in ws], [len(w.points) for w in ws])


def test_batch_matches_oracle_per_circuit(env):
    import torch
    ctx, s = env
    ws = W.batch_config(P_cap=24)
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    for i in range(0, len(ws), 3):
        w = ws[i]
        f, g, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
        e = dict(f=rel(t2n(bufs[i]["out"]), f), g=rel(t2n(bufs[i]["tan"]), g),
                 loss=rel(t2n(bufs[i]["loss"]), [L]), grad=rel(t2n(bufs[i]["grad"]), grad))
        report(f"batch {w.name}", **e)
        for k, v in e.items():
            assert v < TOL, (w.name, k, v)


def test_batch_with_an_empty_member(env):
    """A circuit given no points sits between circuits that have points: it gets no work item,
    its loss and gradient are the empty sums (zero), and its neighbours match the oracle."""
    import torch
    from copy import deepcopy
    ctx, s = env
    ws = [deepcopy(w) for w in W.batch_config(P_cap=40)[:4]]
    ws[1].points = ws[1].points[:0]
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    assert float(t2n(bufs[1]["loss"])[0]) == 0.0
    assert np.all(t2n(bufs[1]["grad"]) == 0.0)
    for i in (0, 2, 3):
        w = ws[i]
        f, g, L, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
        e = dict(f=rel(t2n(bufs[i]["out"]), f), g=rel(t2n(bufs[i]["tan"]), g),
                 loss=rel(t2n(bufs[i]["loss"]), [L]), grad=rel(t2n(bufs[i]["grad"]), grad))
        report(f"batch with empty member: {w.name}", **e)
        for k, v in e.items():
            assert v < TOL, (w.name, k, v)


def test_batch_matches_single_circuit_path(env):
    import torch
    from paper_2506_23246_amd.api import Circuit
    ctx, s = env
    ws = W.batch_config(P_cap=300)
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc())
        singles = [Circuit(ctx, w.circuit).maxwell(w.params, w.points, w.loss) for w in ws]
    s.synchronize()
    for i, w in enumerate(ws):
        for key in ("out", "tan"):   # same per-point kernels: identical
            assert np.array_equal(t2n(bufs[i][key]), t2n(singles[i][key])), (w.name, key)
        assert rel(t2n(bufs[i]["grad"]), t2n(singles[i]["grad"])) < 1e-6
        assert rel(t2n(bufs[i]["loss"]), t2n(singles[i]["loss"])) < 1e-6


def test_batch_autotuned_grid_matches_oracle(env):
    """QP_FLAG_TUNE times persistent grid sizes and class grids (split or stacked) once; the tuned
    batch still matches the oracle per circuit."""
    import torch
    from paper_2506_23246_amd import _lib as L
    ctx, s = env
    ws = W.batch_config(P_cap=64)
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc(), flags=L.QP_FLAG_TUNE)
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    for i in range(1, len(ws), 4):
        w = ws[i]
        f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
        e = dict(f=rel(t2n(bufs[i]["out"]), f), g=rel(t2n(bufs[i]["tan"]), g),
                 loss=rel(t2n(bufs[i]["loss"]), [Lo]), grad=rel(t2n(bufs[i]["grad"]), grad))
        report(f"tuned batch {w.name} grids={b.info(5)},{b.info(6)}", **e)
        for k, v in e.items():
            assert v < TOL, (w.name, k, v)


def test_batch_graph_replays_match_eager(env):
    """Capture once, replay several times with new parameters written in place and eager work
    and synchronisations between the replays; every replay equals an eager run."""
    import torch
    ctx, s = env
    ws = W.batch_config(P_cap=200)
    b = _batch(ctx, ws)
    rng = np.random.default_rng(5)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    eager0 = [{k: t2n(v).copy() for k, v in bb.items() if v is not None} for bb in bufs]
    for rep in range(3):
        with torch.cuda.stream(s):
            b.run(arr, W.MaxwellDesc(), graph=True)
        s.synchronize()
        got = [{k: t2n(v).copy() for k, v in bb.items() if v is not None} for bb in bufs]
        for i in range(len(ws)):
            for k in got[i]:
                if k == "params" or k == "points":
                    continue
                assert np.array_equal(got[i][k], eager0[i][k]), (rep, i, k)
        _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
    assert b.info(3) == 1
    # new parameters in place: replay == eager on the new values
    with torch.cuda.stream(s):
        for i, w in enumerate(ws):
            bufs[i]["params"].copy_(torch.tensor(rng.uniform(0, 6.28, w.circuit.n_params), dtype=torch.float32))
        b.run(arr, W.MaxwellDesc(), graph=True)
    s.synchronize()
    g1 = [t2n(bb["grad"]).copy() for bb in bufs]
    with torch.cuda.stream(s):
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    for i in range(len(ws)):
        assert np.array_equal(g1[i], t2n(bufs[i]["grad"]))
    w = ws[4]
    _, _, L, grad = O.maxwell_eval(w.circuit, t2n(bufs[4]["params"]), w.points, w.loss)
    assert rel(g1[4], grad) < TOL


def test_full_size_batch_sampled_outputs(env):
    """The full uneven batch (about half a million points): sampled outputs against the oracle,
    finite loss and gradients, deterministic repeat."""
    import torch
    ctx, s = env
    ws = W.batch_config()
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    first = [t2n(bb["grad"]).copy() for bb in bufs]
    with torch.cuda.stream(s):
        b.run(arr, W.MaxwellDesc())
    s.synchronize()
    for i, w in enumerate(ws):
        assert np.array_equal(first[i], t2n(bufs[i]["grad"]))
        assert np.all(np.isfinite(first[i]))
        if i % 4 == 0:
            idx = np.linspace(0, len(w.points) - 1, 4).astype(int)
            f, g = O.simulate(w.circuit, w.params, w.points[idx])
            e = rel(t2n(bufs[i]["out"])[idx], f), rel(t2n(bufs[i]["tan"])[idx], g)
            report(f"full batch {w.name} P={len(w.points)}", f=e[0], g=e[1])
            assert e[0] < TOL and e[1] < TOL


@pytest.mark.parametrize("cls", ["low", "high"])
def test_batch_with_one_class_only(env, cls):
    """Every member in one qubit-count class (3..8 or 9..11): one kernel on the whole grid, before
    and after tuning, equal to the single-circuit path."""
    import torch
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Circuit
    ctx, s = env
    ws = [w for w in W.batch_config(P_cap=200) if (w.circuit.n <= 8) == (cls == "low")][:6]
    assert ws
    b = _batch(ctx, ws)
    assert b.info(4) == (b.info(1) if cls == "low" else 0)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        for flags in (0, L.QP_FLAG_TUNE):
            b.run(arr, W.MaxwellDesc(), flags=flags)
            singles = [Circuit(ctx, w.circuit).maxwell(w.params, w.points, w.loss) for w in ws]
            s.synchronize()
            for i, w in enumerate(ws):
                for key in ("out", "tan"):
                    assert np.array_equal(t2n(bufs[i][key]), t2n(singles[i][key])), (w.name, key)
                assert rel(t2n(bufs[i]["grad"]), t2n(singles[i]["grad"])) < 1e-6
                assert rel(t2n(bufs[i]["loss"]), t2n(singles[i]["loss"])) < 1e-6
    assert b.info(2) % ctx.cu_count == 0


def _mixed_members():
    """Members of every work-item segment: RFF encodings, Cross-Mesh CRZ phase stages in the low,
    high and 12-qubit classes, a 12-qubit ring circuit, and plain low and high members; point
    counts that span several tiles with a ragged last one (one point per tile at 12 qubits)."""
    import math
    rng = np.random.default_rng(77)

    def rff_enc(n, F=16):
        B = rng.standard_normal((F, 3)).astype(np.float32)
        Wm = (rng.standard_normal((n, 2 * F)) / math.sqrt(2 * F)).astype(np.float32)
        return W.Encoding(kind=W.ENC_RFF, gate=W.ENC_RY, scale=W.SCALE_NONE, rff_B=B, rff_W=Wm)

    circs = [
        (W.layered(5, 2, "rot", lambda l: W.ring(5, W.CZ, 1 + l % 2), name="rff_5q2l", enc=rff_enc(5)), 301),
        (W.cross_mesh(4, 2, rot="x"), 203),
        (W.layered(6, 3, "xyz", lambda l: W.ring(6, W.CNOT, 1), name="ring_6q3l"), 190),
        (W.cross_mesh(9, 1, rot="xz"), 11),
        (W.layered(10, 2, "xyz", lambda l: W.ring(10, W.CZ, 1), name="ring_10q2l",
                   enc=rff_enc(10)), 13),
        (W.layered(12, 2, "xyz", lambda l: W.ring(12, W.CNOT, 1), name="ring_12q2l"), 5),
        (W.cross_mesh(12, 1, rot="x"), 3),
    ]
    out = []
    for c, P in circs:
        pts = W.uniform_points(rng, P)
        prm = W.uniform_params(rng, c.n_params)
        out.append(W.Workload(c.name, c, prm, pts, W.MaxwellDesc(W.LOSS_DIEL_SPLIT, 4.0, 0.0)))
    return out


def test_batch_mixed_segments_match_oracle_and_single_path(env):
    """RFF encodings, CRZ phase stages and 12-qubit members in one batch: every member against the
    oracle (split dielectric loss), outputs bitwise equal to the single-circuit path."""
    import torch
    from paper_2506_23246_amd.api import Circuit
    ctx, s = env
    ws = _mixed_members()
    b = _batch(ctx, ws)
    assert b.info(7) > 0 and b.info(8) > 0   # 12-qubit items; items of CRZ circuits
    loss = ws[0].loss
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, loss)
        singles = [Circuit(ctx, w.circuit).maxwell(w.params, w.points, loss) for w in ws]
    s.synchronize()
    for i, w in enumerate(ws):
        f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, loss)
        e = dict(f=rel(t2n(bufs[i]["out"]), f), g=rel(t2n(bufs[i]["tan"]), g),
                 loss=rel(t2n(bufs[i]["loss"]), [Lo]), grad=rel(t2n(bufs[i]["grad"]), grad))
        report(f"mixed batch {w.name} P={len(w.points)}", **e)
        for k, v in e.items():
            assert v < TOL, (w.name, k, v)
        for key in ("out", "tan"):
            assert np.array_equal(t2n(bufs[i][key]), t2n(singles[i][key])), (w.name, key)
        assert rel(t2n(bufs[i]["grad"]), t2n(singles[i]["grad"])) < 1e-6
        assert rel(t2n(bufs[i]["loss"]), t2n(singles[i]["loss"])) < 1e-6


def test_batch_mixed_segments_graph_replay(env):
    """The table and RFF-angle kernels of CRZ and RFF members sit inside the captured graph: a
    replay after new parameters and points are written in place equals an eager run."""
    import torch
    ctx, s = env
    ws = _mixed_members()
    b = _batch(ctx, ws)
    loss = ws[0].loss
    rng = np.random.default_rng(9)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, loss, graph=True)
        for i, w in enumerate(ws):
            bufs[i]["params"].copy_(torch.tensor(rng.uniform(0, 6.28, w.circuit.n_params), dtype=torch.float32))
            bufs[i]["points"].copy_(torch.tensor(rng.uniform(-1, 1, (len(w.points), 3)), dtype=torch.float32))
        b.run(arr, loss, graph=True)
    s.synchronize()
    got = [{k: t2n(bufs[i][k]).copy() for k in ("out", "tan", "loss", "grad")} for i in range(len(ws))]
    with torch.cuda.stream(s):
        b.run(arr, loss)
    s.synchronize()
    for i in range(len(ws)):
        for k in got[i]:
            assert np.array_equal(got[i][k], t2n(bufs[i][k])), (ws[i].name, k)
    i = 1   # a CRZ member against the oracle on the new values
    _, _, Lo, grad = O.maxwell_eval(ws[i].circuit, t2n(bufs[i]["params"]), t2n(bufs[i]["points"]), loss)
    assert rel(got[i]["grad"], grad) < TOL and rel(got[i]["loss"], [Lo]) < TOL


def test_batch_rejects_angle_encoding(env):
    """qp_batch_io carries no per-point angles: an angle-given circuit is refused at compile time."""
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import Batch
    ctx, _ = env
    c = W.paper_context_circuit()
    with pytest.raises(L.QPError, match="angle-given encoding not batched"):
        Batch(ctx, [c], [16])


@pytest.mark.parametrize("kind,loss_sum", [(W.LOSS_DIEL_INTUITIVE, False), (W.LOSS_VACUUM, True)])
def test_batch_mixed_segments_other_losses(env, kind, loss_sum):
    """The mixed batch under the intuitive dielectric loss, and under the vacuum loss with
    QP_FLAG_LOSS_SUM (plain sums: the oracle's mean loss and gradient times the member's point
    count), against the oracle member by member."""
    import torch
    from paper_2506_23246_amd import _lib as L
    ctx, s = env
    ws = _mixed_members()
    loss = W.MaxwellDesc(kind, 4.0, 0.0)
    b = _batch(ctx, ws)
    with torch.cuda.stream(s):
        arr, bufs = b.io([w.params for w in ws], [w.points for w in ws])
        b.run(arr, loss, flags=L.QP_FLAG_LOSS_SUM if loss_sum else 0)
    s.synchronize()
    for i, w in enumerate(ws):
        f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, loss)
        scale = len(w.points) if loss_sum else 1.0
        e = dict(f=rel(t2n(bufs[i]["out"]), f), g=rel(t2n(bufs[i]["tan"]), g),
                 loss=rel(t2n(bufs[i]["loss"]), [Lo * scale]), grad=rel(t2n(bufs[i]["grad"]), grad * scale))
        report(f"mixed batch kind={kind} sum={loss_sum} {w.name}", **e)
        for k, v in e.items():
            assert v < TOL, (w.name, k, v)
