"""Builds libqpinn.so (the C-ABI library) in-tree for gfx950 with hipcc.

Every HIP unit is compiled with packed-FP32 instructions disabled; objects go to
``paper_2506_23246_amd/_build`` and the library to ``paper_2506_23246_amd/libqpinn.so``.
Run ``python -m paper_2506_23246_amd.build`` (add ``--incremental`` to reuse up-to-date objects).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqpinn.so")
ARCH = "gfx950"   # the kernels use gfx950 cross-lane swaps and the CDNA4 LDS layout
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only within one source expression, as written, so the
# rounding of every kernel's arithmetic follows the source and not the surrounding code (kernel
# variants that share per-point code give bitwise-equal results).
HIP_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17", "-Wno-unused-command-line-argument",
             "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CPP_FLAGS = ["-O2", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-variable",
             "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _sources():
    hip = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    cpp = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    return hip, cpp


def _headers_mtime():
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(PKG, "..", "include", "*.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src, incremental, hmt):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(src), hmt):
            return obj, ""
    flags = HIP_FLAGS if src.endswith(".hip") else CPP_FLAGS
    cmd = [HIPCC, "-c", *flags, src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(incremental: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = _sources()
    hmt = _headers_mtime()
    jobs = jobs or min(16, os.cpu_count() or 4)
    srcs = hip + cpp
    # the heaviest units first so the pool stays busy
    srcs.sort(key=lambda s: (0 if "batch" in s else 1 if "fused_n" in s else 2, s))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, incremental, hmt): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, log = f.result()
            objs.append(obj)
            if verbose:
                print("built", os.path.basename(obj), flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *sorted(objs), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    lib = build(incremental="--incremental" in sys.argv, verbose=True)
    print(lib)
