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
    print(json.dumps({"tuned": [c.info(8), c.info(9)]}), flush=True)
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
