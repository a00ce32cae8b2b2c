"""Build the gfx950 shared library ``libtc2.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtc2.so")
SOURCES = ["tc2_kernels.hip", "tc2_tile.hip", "tc2_mlp.hip", "tc2_runtime.hip", "tc2_dense.hip",
           "tc2_lowdin.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# the dense O(N^3) path: eigenpairs (rocSOLVER) and products (rocBLAS)
LIBS = ["-lrocsolver", "-lrocblas"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into ``libtc2.so``; returns its path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtc2.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
