"""Host-side parts of bench.py (CPU only): the one-GPU guard, the flop counts behind the roofline
figure and the lookup of recorded HBM traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("F,n", [(1, 0), (3, 2), (96, 12), (30, 6)])
def test_algorithmic_flops_count_four_eight_and_four_statevectors(F, n):
    # forward: psi + 3 tangents; adjoint: uncompute psi + pull back lambda for 4 each; gate
    # statistics priced as 4 more statevectors; 16 flop per amplitude per statevector and gate
    # (two outputs of 4 real products each, counted as 8 FMA slots of 2 flop)
    per_sv = 2 * 4 * 2
    assert bench.flops_per_point(F, n) == F * (2 ** n) * (4 + 8 + 4) * per_sv


def test_executed_flops_closed_forms():
    # one gate on one amplitude: a real part is 1 mul + 3 fma = 7 flop, a complex output 14,
    # times 4 + 8 statevectors, plus the 3-component statistic over 4 statevector pairs at 4 fma
    # per amplitude pair (two amplitudes)
    assert bench.executed_flops_per_point(1, 0) == 14 * (4 + 8) + 3 * 4 * 4 * 2 // 2
    assert bench.executed_flops_per_point(96, 12) == 96 * 216 * 4096
    # a gate folded into the encoding keeps only its statistic
    assert bench.executed_flops_per_point(5, 3, 5) == 5 * 48 * 8
    assert bench.executed_flops_per_point(96, 12, 12) < bench.executed_flops_per_point(96, 12)


def test_recorded_traffic_needs_kernel_workload_and_sources_to_match(tmp_path, monkeypatch):
    rec = {"kernel": "k_fused", "workload": "w12", "traffic_bytes_per_launch": 1234,
           "sources_sha256": "digest-a"}
    (tmp_path / "k_fused_w12_hbm_counters.md").write_text(
        "# counters\n| a | b |\n" + json.dumps(rec) + "\n" + "{not json\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda kernel="k_fused": "digest-a")
    value, src = bench.recorded_traffic("k_fused", "w12")
    assert value == 1234 and src.endswith("k_fused_w12_hbm_counters.md")
    assert bench.recorded_traffic("k_batch", "w12") == (None, None)
    assert bench.recorded_traffic("k_fused", "w6") == (None, None)
    monkeypatch.setattr(bench, "sources_digest", lambda kernel="k_fused": "digest-b")
    assert bench.recorded_traffic("k_fused", "w12") == (None, None)


def test_sources_digest_covers_the_library_sources():
    d = bench.sources_digest()
    assert len(d) == 64 and int(d, 16) >= 0
    assert d == bench.sources_digest("k_fused")
    assert bench.sources_digest("k_batch") != d
    for kernel, pats in bench.KERNEL_SOURCES.items():
        import glob
        for pat in pats:
            assert glob.glob(os.path.join(ROOT, "paper_2506_23246_amd", "csrc", pat)), (kernel, pat)
