"""The fused Maxwell step captured in a HIP graph (through torch.cuda.CUDAGraph on a dedicated
stream): every replay, with eager work and synchronisations in between, reproduces the eager
result bitwise (the step launches kernels only, no memset or allocation nodes)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import t2n

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,P", [(1, 1000), (2, 300), (4, 12)])
def test_graph_replays_match_eager(k, P):
    import torch
    from paper_2506_23246_amd.api import Circuit, Context
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream()
    ctx = Context(0, stream=s)
    w = W.config(k, P=P)
    c = Circuit(ctx, w.circuit)
    prm = torch.tensor(np.asarray(w.params, np.float32), device=dev)
    pts = torch.tensor(np.asarray(w.points, np.float32), device=dev)
    torch.cuda.synchronize()
    bufs = {"out": torch.empty((P, 3), dtype=torch.float32, device=dev),
            "tan": torch.empty((P, 3, 3), dtype=torch.float32, device=dev),
            "loss": torch.empty(1, dtype=torch.float64, device=dev),
            "grad": torch.empty(w.circuit.n_params, dtype=torch.float32, device=dev)}
    with torch.cuda.stream(s):
        c.maxwell(prm, pts, w.loss, bufs=bufs)
    s.synchronize()
    ref = {key: t2n(v).copy() for key, v in bufs.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        c.maxwell(prm, pts, w.loss, bufs=bufs)
    for rep in range(3):
        for v in bufs.values():          # eager work between replays: poison the outputs
            v.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        s.synchronize()
        for key, v in bufs.items():
            assert np.array_equal(t2n(v), ref[key]), (rep, key)
