"""Build librve.so in-tree with hipcc for gfx950.

    python -m paper_1903_12227_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("kernels_vec.hip", "kernels_gemm.hip", "kernels_3d.hip", "kernels_small.hip", "kernels_sample.hip", "kernels_dos.hip", "rve_api.hip")
OUT = os.path.join(HERE, "librve.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-fPIC", "-shared", "-std=c++17", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = OUT + ".tmp"
    cmd = [hipcc(), *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building librve.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
