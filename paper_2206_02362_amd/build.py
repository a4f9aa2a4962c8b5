"""Build the HIP library libfwime.so for gfx950 in-tree (hipcc, no JIT cache).

Usage: python -m paper_2206_02362_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwime.so")
SOURCES = ["kernels_step.hip", "kernels_step2.hip", "kernels_ext.hip", "kernels_vec.hip", "kernels_spline.hip", "runtime.hip"]

# Packed FP32 instructions are disabled on purpose: plain scalar FP32 only.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, src.replace(".hip", ".o")) for src in SOURCES]
    # one hipcc per translation unit, compiled concurrently
    from concurrent.futures import ThreadPoolExecutor
    jobs = min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, [hipcc, *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
                  for src, obj in zip(SOURCES, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
