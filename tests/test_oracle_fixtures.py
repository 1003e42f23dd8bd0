"""The stored oracle results (tests/golden/*.npz) and the process-parallel oracle driver (CPU).

* The parallel driver returns what the serial oracle returns (chunking only splits the points;
  the loss weights are taken over the whole set).
* Each stored set loads without pickled objects, has the shapes of its workload, agrees with a
  fresh serial oracle evaluation on a few of its points, and (where every point is stored) holds
  the loss that the oracle's loss function gives on the stored tangents.
"""
import numpy as np
import pytest

import workloads as W
from oracle import parallel as OP
from oracle import qpinn_oracle as O
from tests.golden.make_oracle_fixtures import SETS, load


def test_parallel_driver_matches_serial_oracle():
    w = W.config(2, P=40)        # RFF, strided CZ, split dielectric loss (weights over the set)
    with OP.Pool(2) as pool:
        f, g, loss, grad = OP.maxwell_eval(pool, w.circuit, w.params, w.points, w.loss, chunk=7)
    f0, g0, loss0, grad0 = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    assert np.allclose(f, f0, rtol=0, atol=1e-13) and np.allclose(g, g0, rtol=0, atol=1e-12)
    assert abs(loss - loss0) <= 1e-12 * abs(loss0)
    assert np.allclose(grad, grad0, rtol=0, atol=1e-12 * np.abs(grad0).max())


@pytest.mark.parametrize("name", list(SETS))
def test_stored_set_is_the_oracle(name):
    w = SETS[name]()
    ref = load(name)
    P, m, K = len(w.points), len(w.circuit.out_qubits), w.circuit.n_params
    assert int(ref["P"]) == P and str(ref["workload"]) == w.name
    idx = ref["idx"]
    S = len(idx)
    assert idx[0] == 0 and idx[-1] == P - 1 and np.all(np.diff(idx) > 0)
    assert ref["f"].shape == (S, m) and ref["g"].shape == (S, m, 3) and ref["grad"].shape == (K,)
    if S == P:
        assert float(ref["loss"]) == pytest.approx(O.maxwell_loss(ref["g"], w.points, w.loss), rel=1e-14)
    # a few stored points (both ends) recomputed serially
    pick = np.array([0, 1, S // 2, S - 1])
    f, g = O.simulate(w.circuit, w.params, w.points[idx[pick]])
    assert np.allclose(ref["f"][pick], f, rtol=0, atol=1e-13)
    assert np.allclose(ref["g"][pick], g, rtol=0, atol=1e-12)
    assert np.all(np.isfinite(ref["grad"])) and np.linalg.norm(ref["grad"]) > 0
