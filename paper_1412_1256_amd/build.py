"""Build the gfx950 HIP library libpolaris.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpolaris.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled for every device pass
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"--offload-arch={ARCH}"]
SOURCES = ["polaris_kernels.hip", "polaris_backward.hip", "polaris_mfma.hip", "polaris_post.hip", "polaris_fused.hip", "polaris_api.cpp"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (in parallel, at most `jobs` at a time: MAX_JOBS or 8) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(8, int(os.environ.get("MAX_JOBS", "8"))))
    objs, running = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        if len(running) >= jobs:
            _wait(running.pop(0))
        running.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    for r in running:
        _wait(r)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def _wait(r) -> None:
    proc, src = r
    if proc.wait() != 0:
        raise subprocess.CalledProcessError(proc.returncode, f"hipcc {src}")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
