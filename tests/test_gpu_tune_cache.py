"""The autotuner's cache file (QP_TUNE_CACHE) round trip: a tuned run records its launch choice,
and a later process that compiles the same circuit shape starts with the cached choice.

The library reads the file once per process, so each side runs in a child process of its own
(one at a time; each holds the GPU only for its few calls)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[2])
import workloads as W
from paper_2506_23246_amd import _lib as L
from paper_2506_23246_amd.api import Circuit, Context
ctx = Context(0)
w = W.config(1, P=4096)
c = Circuit(ctx, w.circuit)
print(json.dumps({"compiled": [c.info(8), c.info(9)]}), flush=True)
if sys.argv[1] == "tune":
    c.maxwell(w.params, w.points, w.loss, flags=L.QP_FLAG_TUNE)
    print(json.dumps({"tuned": [c.info(8), c.info(9)], "dense": c.info(13)}), flush=True)
if sys.argv[1] == "dense":
    import numpy as np
    from oracle import qpinn_oracle as O
    t = lambda x: x.detach().cpu().numpy().copy()
    rel = lambda a, b: float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))
    routed = c.info(13)
    r1 = {k: t(v) for k, v in c.maxwell(w.params, w.points, w.loss).items()}
    r2 = {k: t(v) for k, v in c.maxwell(w.params, w.points, w.loss, flags=L.QP_FLAG_DENSE_MFMA).items()}
    f, g, Lo, grad = O.maxwell_eval(w.circuit, w.params, w.points, w.loss)
    c.set_launch(4, 2)
    r3 = {k: t(v) for k, v in c.maxwell(w.params, w.points, w.loss).items()}
    print(json.dumps({"routed": routed, "after_set_launch": c.info(13),
                      "same_as_dense": all(np.array_equal(r1[k], r2[k]) for k in ("out", "tan", "loss", "grad")),
                      "fused_differs": not np.array_equal(r3["tan"], r2["tan"]),
                      "err": [rel(r1["out"], f), rel(r1["tan"], g), rel(r1["loss"], [Lo]), rel(r1["grad"], grad)],
                      "err_fused": [rel(r3["tan"], g), rel(r3["grad"], grad)]}), flush=True)
"""


def _child(mode, cache):
    env = dict(os.environ)
    env.pop("QP_TUNE_CACHE", None)
    if cache:
        env["QP_TUNE_CACHE"] = str(cache)
    r = subprocess.run([sys.executable, "-c", CHILD, mode, ROOT], capture_output=True, text=True,
                       timeout=180, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    out = {}
    for ln in r.stdout.splitlines():
        if ln.startswith("{"):
            out.update(json.loads(ln))
    return out


def test_cached_choice_applies_at_compile_time(tmp_path):
    cache = tmp_path / "tune.jsonl"
    default = _child("compile", None)["compiled"]
    first = _child("tune", cache)
    assert first["compiled"] == default                  # nothing cached yet
    tuned = first["tuned"]
    lines = [json.loads(ln) for ln in cache.read_text().splitlines()]
    any_keys = [e for e in lines if e["key"].endswith("/any")]
    assert any_keys and [any_keys[-1]["exs"], any_keys[-1]["wg_per_cu"]] == tuned
    assert _child("compile", cache)["compiled"] == tuned
    # a hand-edited entry with another legal shape is what the next compilation starts with
    other = [2, 1] if tuned != [2, 1] else [4, 2]
    e = dict(any_keys[-1], exs=other[0], wg_per_cu=other[1])
    with open(cache, "a") as fh:
        fh.write(json.dumps(e) + "\n")
    assert _child("compile", cache)["compiled"] == other


def test_cached_dense_fusion_width_routes_maxwell_calls(tmp_path):
    """The tuner's fusion-width choice: a tuned run records whether the dense-block path (32x32
    blocks on the matrix cores) beat the fused kernel; a cached entry choosing it (here written by
    hand) makes later Maxwell calls on a compiled circuit take that path, bitwise equal to a call
    forced onto it and within the parity bar of the oracle; an explicit launch shape puts the
    calls back on the fused kernel."""
    cache = tmp_path / "tune.jsonl"
    first = _child("tune", cache)
    lines = [json.loads(ln) for ln in cache.read_text().splitlines()]
    any_keys = [e for e in lines if e["key"].endswith("/any")]
    assert any_keys and any_keys[-1]["dense"] == first["dense"] and first["dense"] in (0, 1)
    with open(cache, "a") as fh:
        fh.write(json.dumps(dict(any_keys[-1], dense=1)) + "\n")
    r = _child("dense", cache)
    assert r["routed"] == 1 and r["after_set_launch"] == 0
    assert r["same_as_dense"] and r["fused_differs"]
    assert max(r["err"]) < 1e-5 and max(r["err_fused"]) < 1e-5, r
