"""Writes the stored oracle results that the multi-tile GPU parity tests compare against.

Every value here comes from the CPU oracle (``oracle/``) evaluated on the seeded inputs of
``workloads.py``; nothing is read from the HIP path.  For each set the file holds the Maxwell
loss over the whole set, its gradient d loss / d params [K], and the outputs f and input tangents g
(float64) at the point indices ``idx``: every point for sets of up to 4096 points, else 4096
indices spread over the set (both ends and the last, ragged tile included), which keeps the
files small; the per-point values do not depend on how points are grouped into tiles.

* ``c5_first4096.npz``  - the first 4096 points of the 12-qubit, 8-layer CNOT-ring vacuum
  workload (the size of its error subsample; sixteen one-point tiles per persistent
  workgroup at the default launch of a 256-CU device);
* ``c3_first16384.npz`` - the first 16384 points of the 8-qubit, 10-layer Rot + strided-CZ
  workload with random Fourier features and the split dielectric loss (four 8-point tiles per
  workgroup);
* ``multitile_4q.npz``  - the 4-qubit, 2-layer circuit at 2 * 65536 + 4096 + 37 points (two
  or three 128-point tiles per workgroup, ragged last tile).

Run from the repository root: ``python tests/golden/make_oracle_fixtures.py [name ...]``.
The oracle is evaluated in parallel over point chunks (``oracle.parallel``); a few minutes on
eight cores.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import parallel as OP  # noqa: E402

SETS = {
    "c5_first4096": lambda: W.config(4, P=4096),
    "c3_first16384": lambda: W.config(2, P=16384),
    "multitile_4q": lambda: W.multitile_config(),
}


def sample_indices(P: int, cap: int = 4096) -> np.ndarray:
    """All indices up to `cap` points, else `cap` indices spread evenly, the last 64 included."""
    if P <= cap:
        return np.arange(P, dtype=np.int64)
    spread = np.linspace(0, P - 65, cap - 64).astype(np.int64)
    return np.unique(np.concatenate([spread, np.arange(P - 64, P, dtype=np.int64)]))


def load(name: str):
    """The stored arrays of one set (no pickled objects are loaded)."""
    with np.load(os.path.join(HERE, name + ".npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def main(names):
    with OP.Pool() as pool:
        for name in names:
            w = SETS[name]()
            t0 = time.time()
            f, g, loss, grad = OP.maxwell_eval(pool, w.circuit, w.params, w.points, w.loss)
            idx = sample_indices(len(w.points))
            np.savez_compressed(os.path.join(HERE, name + ".npz"), idx=idx, f=f[idx], g=g[idx],
                                loss=np.array(loss), grad=grad,
                                P=np.array(len(w.points)), workload=np.array(w.name))
            print(f"{name}: P={len(w.points)} loss={loss:.6e} |grad|={np.linalg.norm(grad):.6e} "
                  f"({time.time() - t0:.0f} s on {pool.workers} workers)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(SETS))
