"""Build the gfx950 shared library ``libtc2.so`` in-tree with hipcc.

Each HIP source is compiled to an object file in its own hipcc process (in
parallel), then the objects are linked into the library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtc2.so")
SOURCES = ["tc2_kernels.hip", "tc2_tile.hip", "tc2_mlp.hip", "tc2_runtime.hip", "tc2_dense.hip",
           "tc2_lowdin.hip", "tc2_measure.hip", "tc2_memory.hip", "tc2_decide.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# the dense O(N^3) path: eigenpairs (rocSOLVER) and products (rocBLAS)
LIBS = ["-lrocsolver", "-lrocblas"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source and link ``libtc2.so``; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, s.replace(".hip", ".o")) for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(cmds)))) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
