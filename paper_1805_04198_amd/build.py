"""Build libeik.so (HIP, gfx950) in-tree, and libeik_ceilings.so, the
measured-ceiling probes the benchmark reports beside the published peaks.

    python -m paper_1805_04198_amd.build

Flags that matter for results: -ffp-contract=off (no fused multiply-add, so
device arithmetic rounds exactly as written), packed FP32 instructions
disabled, denormals kept."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "eik.hip")
OUT_DIR = os.path.join(HERE, "_lib")
OUT = os.path.join(OUT_DIR, "libeik.so")
CEIL_SRC = os.path.join(HERE, "csrc", "ceilings.hip")
CEIL_OUT = os.path.join(OUT_DIR, "libeik_ceilings.so")
ARCH = os.environ.get("EIK_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc, *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    tmp = CEIL_OUT + ".tmp"
    cmd = [hipcc, *FLAGS, CEIL_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CEIL_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
