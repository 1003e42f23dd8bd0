"""Process-parallel driver of the CPU oracle over chunks of collocation points.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` (and the scripts that
write their stored expected values), ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.

Points are independent in every quantity the oracle computes except through the loss weights
(1/P, or 1/N_vac and 1/N_diel for the split dielectric loss), so the full-set evaluation splits
into three phases:

1. forward: f and g per chunk (``qpinn_oracle.simulate``), in parallel;
2. the loss and its seeds W = d loss / d g over the whole set (cheap, in the parent);
3. reverse mode per chunk with that chunk's rows of W (``qpinn_oracle.grad_reverse``), in
   parallel; the chunk gradients are summed in chunk order, so the result does not depend on
   the number of workers.

Nothing of the oracle's arithmetic is changed or reordered inside a chunk.  Each worker runs
single-threaded BLAS (the sparse Kronecker operators used at 10 and 12 qubits are
single-threaded anyway), so the pool size is the number of cores used.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import qpinn_oracle as O


def host_cores(cap: int = 16) -> int:
    """Cores this process may run on (its affinity mask), at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass


def _fwd(args):
    circ, params, pts, ang, jac = args
    return O.simulate(circ, params, pts, ang, jac)


def _rev(args):
    circ, params, pts, ang, jac, wf, wg = args
    return O.grad_reverse(circ, params, pts, wf, wg, ang, jac)


def _chunks(P: int, chunk: int):
    return [(s, min(P, s + chunk)) for s in range(0, P, chunk)]


def _sl(a, s, e):
    return None if a is None else a[s:e]


class Pool:
    """A fork-context process pool with single-threaded BLAS in every worker.

    Workers are forked copies of the caller, so open the pool before the calling process
    initialises a GPU (forking a process that holds a GPU context is not supported)."""

    def __init__(self, workers: int | None = None):
        self.workers = workers or host_cores()
        self._pool = mp.get_context("fork").Pool(self.workers, initializer=_init_worker)

    def map(self, fn, items):
        return self._pool.map(fn, items, chunksize=1)

    def close(self):
        self._pool.close()
        self._pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def default_chunk(n: int) -> int:
    """Points per task: small enough to balance the pool, large enough to amortise the per-task
    operator construction (about 16 points at 12 qubits, where one task takes a few seconds)."""
    return 16 if n >= 12 else 64 if n >= 10 else 256


def simulate(pool: Pool, circ, params, points, angles=None, jac=None, chunk=None):
    """f [P,m] and g [P,m,3] of ``qpinn_oracle.simulate``, chunked over the pool."""
    P = len(points) if points is not None else len(angles)
    chunk = chunk or default_chunk(circ.n)
    parts = pool.map(_fwd, [(circ, params, _sl(points, s, e), _sl(angles, s, e), _sl(jac, s, e))
                            for s, e in _chunks(P, chunk)])
    m = len(circ.out_qubits)
    if not parts:
        return np.zeros((0, m)), np.zeros((0, m, 3))
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def grad_reverse(pool: Pool, circ, params, points, seeds_f, seeds_g, angles=None, jac=None,
                 chunk=None):
    """``qpinn_oracle.grad_reverse`` chunked over the pool; chunk gradients summed in order."""
    P = len(seeds_g)
    chunk = chunk or default_chunk(circ.n)
    parts = pool.map(_rev, [(circ, params, _sl(points, s, e), _sl(angles, s, e), _sl(jac, s, e),
                             _sl(seeds_f, s, e), seeds_g[s:e]) for s, e in _chunks(P, chunk)])
    grad = np.zeros(circ.n_params)
    for p in parts:
        grad += p
    return grad


def maxwell_eval(pool: Pool, circ, params, points, desc, angles=None, jac=None, chunk=None):
    """f, g, loss and d loss / d params over the whole point set (``qpinn_oracle.maxwell_eval``
    in three phases)."""
    f, g = simulate(pool, circ, params, points, angles, jac, chunk)
    loss = O.maxwell_loss(g, points, desc)
    Wg = O.maxwell_seeds(g, points, desc)
    grad = grad_reverse(pool, circ, params, points, None, Wg, angles, jac, chunk)
    return f, g, loss, grad
