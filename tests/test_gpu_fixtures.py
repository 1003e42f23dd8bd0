"""Loss and gradient against stored oracle results where every workgroup runs several tiles.

The fused kernel is persistent: each workgroup walks a range of point tiles and accumulates the
gate statistics and the loss of all of them in FP32 (per-wave LDS slots, then per-workgroup
partials summed in FP64 across workgroups).  These tests run the fused Maxwell step at the
default launch (the one ``bench.py`` times) on point sets large enough that every workgroup of a
256-CU device takes two or more tiles, and compare outputs, tangents, loss and gradient with the
oracle's values stored under ``tests/golden/`` (outputs and tangents at the stored point
indices, loss and gradient over the whole set) (written by ``make_oracle_fixtures.py``, which
calls only the oracle).  Normwise relative error per quantity, bar 1e-5.
"""
import numpy as np
import pytest

from tests.golden.make_oracle_fixtures import SETS, load
from tests.gpu_helpers import TOL, rel, report, t2n

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_23246_amd.api import Context
    assert torch.cuda.is_available()
    return Context(0)


@pytest.mark.parametrize("name", list(SETS))
def test_default_launch_matches_stored_oracle(ctx, name):
    from paper_2506_23246_amd.api import Circuit
    w = SETS[name]()
    ref = load(name)
    P = len(w.points)
    assert int(ref["P"]) == P and str(ref["workload"]) == w.name
    c = Circuit(ctx, w.circuit)
    tiles = -(-P // c.info(7))
    grid = min(tiles, ctx.cu_count * c.info(9))
    print(f"{name}: P={P} tiles={tiles} grid={grid} tiles/workgroup={tiles / grid:.1f}", flush=True)
    if ctx.cu_count >= 256:
        assert tiles >= 2 * grid, "the set must give every workgroup two or more tiles"
    r = c.maxwell(w.params, w.points, w.loss)
    idx = ref["idx"]
    errs = {"f": rel(t2n(r["out"])[idx], ref["f"]), "g": rel(t2n(r["tan"])[idx], ref["g"]),
            "loss": rel(t2n(r["loss"]), [float(ref["loss"])]), "grad": rel(t2n(r["grad"]), ref["grad"])}
    report(f"stored oracle {name}", **errs)
    assert all(v < TOL for v in errs.values()), errs
