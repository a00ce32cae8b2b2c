"""The C ABI called from plain C: tests/c/abi_chain.c, built with
gcc -std=c99 -pedantic -Werror against include/tc2.h and linked with
libtc2.so.  On the CPU the program builds and tc2_setup reports the missing
device; on the GPU its FP64 solve matches the oracle on the same chain."""
import os
import subprocess

import numpy as np
import pytest

from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_chain.c")


def build_caller(tmp_path) -> str:
    libdir = os.path.dirname(T.LIB_PATH)
    assert os.path.exists(T.LIB_PATH), "libtc2.so is not built"
    exe = str(tmp_path / "abi_chain")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.join(ROOT, "include"), "-o", exe, SRC,
                        "-L", libdir, "-ltc2", f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def chain_problem():
    """The chain of abi_chain.c in numpy: 32 atoms, two orbitals each."""
    na, b = 32, 2
    base = np.array([[-0.30, 0.10], [0.05, 0.20]])
    H = np.zeros((na * b, na * b))
    for i in range(na):
        H[i * b:(i + 1) * b, i * b:(i + 1) * b] = np.diag([-1.0, 1.0])
        if i + 1 < na:
            c = base * (1.0 + 0.1 * (i % 3))
            H[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = c
            H[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = c.T
    H1 = np.diag(np.repeat(np.arange(na) - 0.5 * (na - 1), b))
    return H, H1, na, b


def test_c_caller_builds_and_links(tmp_path):
    exe = build_caller(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    # without a GPU, tc2_setup fails with the device error (exit 2)
    assert r.returncode in (0, 2), (r.returncode, r.stdout, r.stderr)
    if r.returncode == 2:
        assert "device" in r.stderr


@pytest.mark.gpu
def test_c_caller_matches_the_oracle(tmp_path):
    exe = build_caller(tmp_path)
    print("  running tests/c/abi_chain.c", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    status, iters, branches, alpha, tr = r.stdout.split()
    H, H1, na, b = chain_problem()
    o = O.tc2_solve(H, [H1], na, b, 1e-10, 1e-10, 100)
    print(f"  C caller: status {status} iters {iters} {branches} alpha {alpha}; "
          f"oracle: iters {o.iters} {o.branches} alpha {o.alpha[0]!r}", flush=True)
    assert branches == o.branches and int(iters) == o.iters
    assert abs(float(alpha) - o.alpha[0]) <= 1e-10 * abs(o.alpha[0])
    assert abs(float(tr) - na) < 1e-8


def test_ctypes_structs_match_the_c_layout(tmp_path):
    # the binding's structures against gcc's layout of include/tc2.h: sizes
    # and the offset of every field of the option, problem and result structs
    import ctypes as C
    structs = {"tc2_options": T.tc2_options, "tc2_problem": T.tc2_problem,
               "tc2_result": T.tc2_result, "tc2_bsr": T.tc2_bsr}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "tc2.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'  printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-o", exe, str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        name, field, val = line.split()
        cls = structs[name]
        want = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, (name, field, int(val), want)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())
