"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects malformed input on the host before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "tc2.h")).read()
    return sorted(set(re.findall(r"TC2_API\s+[\w\s\*]+?\b(tc2_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = T.lib()
    syms = declared_symbols()
    assert set(syms) >= {"tc2_setup", "tc2_run", "tc2_free"}
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (tc2_\w+)", out))
    for s in syms:
        assert s in exported, s
        getattr(lib, s)
    assert set(T.EXPORTED) == set(syms)


def test_strerror_and_version():
    lib = T.lib()
    assert b"gfx950" in lib.tc2_version()
    for code in T.STATUS:
        assert lib.tc2_strerror(code)
    lib.tc2_free(None)  # NULL-safe


def _setup_status(sys_list, **kw):
    try:
        T.Solver(sys_list, **kw).close()
        return 0
    except T.TC2Error as e:
        return e.status


def small():
    return W.config_system("chain64", n=6)


def test_rejects_bad_nocc():
    s = small()
    s.n_occ = s.H.n + 1
    assert _setup_status(s) == -1
    s.n_occ = -1
    assert _setup_status(s) == -1


def test_rejects_bad_eps_tol_iters():
    for attr, val in (("eps", -1.0), ("tol", 0.0), ("max_iter", 0), ("max_iter", 10**6)):
        s = small()
        setattr(s, attr, val)
        assert _setup_status(s) == -1, attr


def test_rejects_unsorted_columns():
    s = small()
    s.H.col = s.H.col.copy()
    r0, r1 = int(s.H.row_ptr[2]), int(s.H.row_ptr[3])
    s.H.col[r0:r1] = s.H.col[r0:r1][::-1]
    assert _setup_status(s) == -1


def test_rejects_nonsymmetric_pattern():
    s = small()
    # drop the (1, 0) entry only
    rp, ci, va = s.H.row_ptr.copy(), s.H.col.copy(), s.H.val.copy()
    p = int(rp[1]) + list(ci[rp[1]:rp[2]]).index(0)
    ci = np.delete(ci, p)
    va = np.delete(va, p, axis=0)
    rp[2:] -= 1
    s.H = W.BSR(s.H.nb, s.H.b, rp, ci, va)
    assert _setup_status(s) == -4


def test_rejects_missing_diagonal():
    s = W.config_system("chain64", n=3, cutoff=0.5)
    H = s.H
    keep = np.array([not (i == 1) for i in range(H.nnzb)])
    rp = np.array([0, 1, 1, 2], dtype=np.int64)
    s.H = W.BSR(3, H.b, rp, H.col[keep], H.val[keep])
    assert _setup_status(s) == -4


def test_rejects_nan():
    s = small()
    s.H.val = s.H.val.copy()
    s.H.val[0, 0, 0] = np.nan
    assert _setup_status(s) == -6


def test_rejects_mismatched_batch():
    a = small()
    b = W.config_system("chain64", n=6, b=5)
    assert _setup_status([a, b]) == -1


def test_rejects_bad_options():
    assert _setup_status(small(), closing_fp64=1) == -1
    assert _setup_status(small(), replay=["SX"]) == -1
    # FP64 sums of the per-block FP32 products exist in the tiled kernel only
    assert _setup_status(small(), precision="fp32", wide=True, kernel="block") == -1
    # updates between two polls of the device-side decisions: 0..TC2_MAX_ITER
    assert _setup_status(small(), device_loop=-1) == -1
    assert _setup_status(small(), device_loop=T.TC2_MAX_ITER + 1) == -1


def test_valid_problem_needs_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _setup_status(small()) == -3


# ---------------------------------------------------------------- dense O(N^3) path
def _dense_status(s):
    try:
        return T.dense_response(s).status
    except T.TC2Error as e:
        return e.status


def test_dense_rejects_malformed_input():
    s = small()
    s.n_occ = s.H.n + 1
    assert _dense_status(s) == -1
    s = small()
    s.H.val = s.H.val.copy()
    s.H.val[0, 0, 0] = np.inf
    assert _dense_status(s) == -6
    s = small()
    rp, ci, va = s.H.row_ptr.copy(), s.H.col.copy(), s.H.val.copy()
    p = int(rp[1]) + list(ci[rp[1]:rp[2]]).index(0)
    rp[2:] -= 1
    s.H = W.BSR(s.H.nb, s.H.b, rp, np.delete(ci, p), np.delete(va, p, axis=0))
    assert _dense_status(s) == -4


def test_dense_rejects_too_large_a_matrix():
    # N = 2501 * 16 > 40000 is refused before any allocation
    nb, b = 2501, 16
    rp = np.arange(nb + 1, dtype=np.int64)
    ci = np.arange(nb, dtype=np.int32)
    va = np.tile(np.eye(b), (nb, 1, 1))
    s = small()
    s.H = W.BSR(nb, b, rp, ci, va)
    s.H1 = []
    s.n_occ = 10
    assert nb * b > T.DENSE_MAX_N
    assert _dense_status(s) == -1


def test_dense_rejects_null_arguments():
    L = T.lib()
    L.tc2_dense_response.restype = C.c_int
    L.tc2_dense_response.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    assert L.tc2_dense_response(None, None, None) == -1


def test_dense_valid_problem_needs_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _dense_status(small()) == -3


# ---------------------------------------------------------------- Loewdin orthogonalisation
def _lowdin_status(S, H, **kw):
    try:
        return T.lowdin(S, H, **kw).status
    except T.TC2Error as e:
        return e.status


def test_lowdin_rejects_malformed_input():
    s = small()
    S = W.make_overlap(s)
    assert _lowdin_status(S, s.H, eps=-1.0) == -1
    assert _lowdin_status(S, s.H, tol=0.0) == -1
    assert _lowdin_status(S, s.H, max_iter=0) == -1
    bad = W.BSR(S.nb, S.b, S.row_ptr, S.col, S.val.copy())
    bad.val[0, 0, 0] = np.nan
    assert _lowdin_status(bad, s.H) == -6
    other = W.config_system("chain64", n=7)
    assert _lowdin_status(S, other.H) == -1          # sizes differ
    # S without its diagonal blocks
    rows = np.repeat(np.arange(S.nb), np.diff(S.row_ptr))
    off = rows != S.col
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[off], minlength=S.nb))]).astype(np.int64)
    assert _lowdin_status(W.BSR(S.nb, S.b, rp, S.col[off], S.val[off]), s.H) == -4


def test_congruence_rejects_mismatched_sizes():
    a, c = small(), W.config_system("chain64", n=7)
    with pytest.raises(T.TC2Error) as ex:
        T.congruence(a.H, c.H)
    assert ex.value.status == -1


def test_lowdin_needs_a_device_and_release_is_null_safe():
    import torch
    L = T.lib()
    L.tc2_bsr_release.restype = None
    L.tc2_bsr_release.argtypes = [C.c_void_p]
    L.tc2_bsr_release(None)
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    s = small()
    assert _lowdin_status(W.make_overlap(s), s.H) == -3
