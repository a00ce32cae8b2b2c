"""ctypes binding of the C ABI in include/tc2.h (argument marshalling only).

Every step of the solve runs in the HIP kernels of ``libtc2.so``; this module
only converts numpy arrays to the C structs and back.  It raises when the
library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Union

import numpy as np

from .workloads import BSR, System

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc2.so")

TC2_MAX_ITER = 200
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "FLOOR_REACHED", -1: "EINVAL", -2: "ENOMEM",
          -3: "EDEVICE", -4: "ENONSYM", -5: "EDEGENERATE", -6: "ENAN", -7: "EOVERFLOW"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
KERNEL = {"tile": 0, "block": 1}
SKIP = {"none": 0, "bound": 1, "mlp": 2}


class tc2_bsr(C.Structure):
    _fields_ = [("nb", C.c_int32), ("b", C.c_int32), ("row_ptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class tc2_problem(C.Structure):
    _fields_ = [("H", tc2_bsr), ("n_dir", C.c_int32), ("H1", tc2_bsr * 3),
                ("n_occ", C.c_int64), ("eps_drop", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("replay", C.c_char_p),
                ("xyz", C.POINTER(C.c_double))]


class tc2_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("closing_fp64", C.c_int32), ("skip", C.c_int32),
                ("device", C.c_int32), ("export_matrices", C.c_int32), ("verbose", C.c_int32),
                ("profile", C.c_int32), ("numeric_kernel", C.c_int32),
                ("fp64_first", C.c_int32), ("mlp_weights", C.POINTER(C.c_float)),
                ("mlp_threshold", C.c_float), ("log_capacity", C.c_int64),
                ("wide_accumulate", C.c_int32), ("tune", C.c_int32), ("tune_cache", C.c_char_p),
                ("graph", C.c_int32), ("metrics_log", C.c_char_p), ("count_useful", C.c_int32),
                ("mlp_bound_cap", C.c_float), ("mlp_budget", C.c_double),
                ("device_loop", C.c_int32)]


class tc2_result(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int32), ("trace_x1h1", C.c_double * 3),
                ("tr_x0", C.c_double), ("idem_err", C.c_double), ("tr_x1", C.c_double * 3),
                ("e0", C.c_double), ("e1", C.c_double * 3), ("emin", C.c_double),
                ("emax", C.c_double), ("seconds", C.c_double), ("useful_flops", C.c_double),
                ("union_flops", C.c_double),
                ("executed_flops", C.c_double), ("kept_blocks", C.c_int64),
                ("screened_blocks", C.c_int64), ("mlp_skipped_blocks", C.c_int64),
                ("mlp_updates", C.c_int32), ("ms_symbolic", C.c_double), ("ms_numeric", C.c_double),
                ("ms_compact", C.c_double), ("numeric_launches", C.c_int32),
                ("tile_shape", C.c_int32 * 4), ("ms_tune", C.c_double),
                ("useful_flops_kind", C.c_double * 4), ("ms_numeric_kind", C.c_double * 4),
                ("numeric_launches_kind", C.c_int32 * 4), ("graph_updates", C.c_int32),
                ("graph_captures", C.c_int32), ("device_loop_updates", C.c_int32),
                ("nominal_flops", C.c_double),
                ("branches", C.c_char * (TC2_MAX_ITER + 4)),
                ("X0", tc2_bsr), ("X1", tc2_bsr * 3)]


_lib = None


def lib() -> C.CDLL:
    """Load libtc2.so (built in-tree by ``build()``); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_2009_03551_amd.build.build()")
        # PyTorch ships its own HIP runtime and ROCm libraries.  Loaded first, it
        # provides them to libtc2.so as well, so that one runtime serves the
        # process; loaded after libtc2.so had brought in the system copies, its
        # own runtime would find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.tc2_setup.restype = C.c_int
        L.tc2_setup.argtypes = [C.POINTER(tc2_problem), C.c_int32, C.POINTER(tc2_options),
                                C.POINTER(C.c_void_p)]
        L.tc2_run.restype = C.c_int
        L.tc2_run.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(tc2_result)]
        L.tc2_free.restype = None
        L.tc2_free.argtypes = [C.c_void_p]
        L.tc2_strerror.restype = C.c_char_p
        L.tc2_strerror.argtypes = [C.c_int]
        L.tc2_version.restype = C.c_char_p
        L.tc2_version.argtypes = []
        L.tc2_trim_memory.restype = C.c_int
        L.tc2_trim_memory.argtypes = [C.c_int32]
        _lib = L
    return _lib


EXPORTED = ("tc2_setup", "tc2_run", "tc2_advance", "tc2_free", "tc2_strerror", "tc2_version",
            "tc2_export_rows", "tc2_iterate_size", "tc2_export_entries", "tc2_compare_entries",
            "tc2_mlp_forward", "tc2_mlp_grad", "tc2_mlp_train", "tc2_log_copy",
            "tc2_dense_response", "tc2_lowdin", "tc2_congruence", "tc2_bsr_release",
            "tc2_lowdin_response", "tc2_congruence_response", "tc2_mlp_grad_noalloc",
            "tc2_trim_memory")

MLP_IN, MLP_PARAMS = 8, 4801


class tc2_progress(C.Structure):
    _fields_ = [("updates", C.c_int32), ("solves_completed", C.c_int32),
                ("solve_open", C.c_int32), ("useful_flops", C.c_double),
                ("executed_flops", C.c_double)]


class tc2_mlp_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("device", C.c_int32)]


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def mlp_forward(theta, X, device: int = 0) -> np.ndarray:
    """Logits of the skip network for rows of X (n x 8), on the device."""
    th, X = _f32(theta, (MLP_PARAMS,)), _f32(X, (-1, MLP_IN))
    out = np.empty(X.shape[0], dtype=np.float32)
    L = lib()
    L.tc2_mlp_forward.restype = C.c_int
    st = L.tc2_mlp_forward(_fptr(th), _fptr(X), C.c_int64(X.shape[0]), C.c_int32(device), _fptr(out))
    if st != 0:
        raise TC2Error(st, "tc2_mlp_forward")
    return out


def mlp_grad(theta, X, y, device: int = 0):
    """(gradient, loss) of the mean binary cross-entropy on logits."""
    th, X, y = _f32(theta, (MLP_PARAMS,)), _f32(X, (-1, MLP_IN)), _f32(y, (-1,))
    g = np.empty(MLP_PARAMS, dtype=np.float32)
    loss = C.c_double()
    L = lib()
    L.tc2_mlp_grad.restype = C.c_int
    st = L.tc2_mlp_grad(_fptr(th), _fptr(X), _fptr(y), C.c_int64(X.shape[0]), C.c_int32(device),
                        _fptr(g), C.byref(loss))
    if st != 0:
        raise TC2Error(st, "tc2_mlp_grad")
    return g, loss.value


MLP_NOALLOC_MAX_N = 65536


def mlp_grad_noalloc(theta_ptr: int, x_ptr: int, y_ptr: int, n: int, grad_ptr: int,
                     loss_ptr: int, stream: Optional[int] = None) -> None:
    """tc2_mlp_grad_noalloc on device pointers (ints, e.g. tensor data_ptr()):
    gradient and mean loss written to grad_ptr / loss_ptr asynchronously on
    ``stream``; nothing is allocated."""
    L = lib()
    L.tc2_mlp_grad_noalloc.restype = C.c_int
    L.tc2_mlp_grad_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
    st = L.tc2_mlp_grad_noalloc(C.c_void_p(theta_ptr), C.c_void_p(x_ptr), C.c_void_p(y_ptr),
                                C.c_int64(n), C.c_void_p(stream) if stream else None,
                                C.c_void_p(grad_ptr), C.c_void_p(loss_ptr))
    if st != 0:
        raise TC2Error(st, "tc2_mlp_grad_noalloc")


def mlp_train(X, y, theta0, epochs: int = 10, batch: int = 4096, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8, device: int = 0):
    """Train on the device with Adam; returns (theta, loss per epoch)."""
    th = _f32(theta0, (MLP_PARAMS,)).copy()
    X, y = _f32(X, (-1, MLP_IN)), _f32(y, (-1,))
    losses = np.zeros(epochs, dtype=np.float64)
    o = tc2_mlp_train_opts(epochs, batch, lr, beta1, beta2, adam_eps, device)
    L = lib()
    L.tc2_mlp_train.restype = C.c_int
    st = L.tc2_mlp_train(_fptr(X), _fptr(y), C.c_int64(X.shape[0]), C.byref(o), _fptr(th),
                         losses.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise TC2Error(st, "tc2_mlp_train")
    return th, losses


class TC2Error(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().tc2_strerror(status).decode()
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")
        self.status = status


@dataclass
class Result:
    status: int
    iters: int
    branches: str
    alpha: List[float]
    tr_x0: float
    idem_err: float
    tr_x1: List[float]
    e0: float
    e1: List[float]
    emin: float
    emax: float
    seconds: float
    useful_flops: float
    executed_flops: float
    kept_blocks: int = 0
    screened_blocks: int = 0
    mlp_skipped_blocks: int = 0
    ms_symbolic: float = 0.0
    ms_numeric: float = 0.0
    ms_compact: float = 0.0
    numeric_launches: int = 0
    tile_shape: List[int] = field(default_factory=list)
    ms_tune: float = 0.0
    useful_flops_kind: List[float] = field(default_factory=list)
    ms_numeric_kind: List[float] = field(default_factory=list)
    numeric_launches_kind: List[int] = field(default_factory=list)
    graph_updates: int = 0
    X0: Optional[BSR] = None
    X1: List[BSR] = field(default_factory=list)
    nominal_flops: float = 0.0
    union_flops: float = 0.0
    graph_captures: int = 0
    mlp_updates: int = 0
    device_loop_updates: int = 0

    @property
    def status_name(self) -> str:
        return STATUS.get(self.status, str(self.status))


def _c_bsr(m: BSR, keep: list) -> tc2_bsr:
    rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(m.col, dtype=np.int32)
    va = np.ascontiguousarray(m.val, dtype=np.float64)
    keep += [rp, ci, va]
    return tc2_bsr(m.nb, m.b, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                   ci.ctypes.data_as(C.POINTER(C.c_int32)),
                   va.ctypes.data_as(C.POINTER(C.c_double)))


def _py_bsr(m: tc2_bsr) -> BSR:
    nb, b = m.nb, m.b
    rp = np.ctypeslib.as_array(m.row_ptr, shape=(nb + 1,)).copy()
    nnz = int(rp[-1])
    ci = np.ctypeslib.as_array(m.col, shape=(max(nnz, 1),))[:nnz].copy()
    va = np.ctypeslib.as_array(m.val, shape=(max(nnz * b * b, 1),))[:nnz * b * b].copy()
    return BSR(nb, b, rp, ci, va.reshape(nnz, b, b))


class Solver:
    """A prepared context (``tc2_setup``) that can be run repeatedly."""

    def __init__(self, systems: Union[System, Sequence[System]], precision: str = "fp64",
                 closing_fp64: int = 0, export: bool = True, device: int = 0,
                 replay: Optional[Sequence[Optional[str]]] = None, verbose: bool = False,
                 profile: bool = False, kernel: str = "tile", use_xyz: bool = True,
                 fp64_first: int = 0, skip: str = "none", mlp_weights=None,
                 mlp_threshold: float = 0.99, log_capacity: int = 0, wide: bool = False,
                 tune: bool = False, tune_cache: Optional[str] = None, graph: bool = False,
                 count_useful: bool = False, metrics_log: Optional[str] = None,
                 mlp_bound_cap: float = 0.0, mlp_budget: float = 0.0, device_loop: int = 0):
        if isinstance(systems, System):
            systems = [systems]
        self.systems = list(systems)
        self._keep: list = []
        n = len(self.systems)
        probs = (tc2_problem * n)()
        for k, s in enumerate(self.systems):
            p = probs[k]
            p.H = _c_bsr(s.H, self._keep)
            p.n_dir = len(s.H1)
            for d, h1 in enumerate(s.H1):
                p.H1[d] = _c_bsr(h1, self._keep)
            p.n_occ = int(s.n_occ)
            p.eps_drop = float(s.eps)
            p.tol = float(s.tol)
            p.max_iter = int(s.max_iter)
            rep = replay[k] if replay is not None else None
            if rep:
                rb = rep.encode()
                self._keep.append(rb)
                p.replay = rb
            else:
                p.replay = None
            if use_xyz and s.xyz is not None:
                xyz = np.ascontiguousarray(s.xyz, dtype=np.float64)
                self._keep.append(xyz)
                p.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
        self.n_dir = len(self.systems[0].H1)
        wptr = None
        if mlp_weights is not None:
            w = _f32(mlp_weights, (MLP_PARAMS,))
            self._keep.append(w)
            wptr = _fptr(w)
        opts = tc2_options(PRECISION[precision], int(closing_fp64), SKIP[skip], int(device),
                           1 if export else 0, 1 if verbose else 0, 1 if profile else 0,
                           KERNEL[kernel], int(fp64_first), wptr, float(mlp_threshold),
                           int(log_capacity), 1 if wide else 0, 1 if tune else 0,
                           tune_cache.encode() if tune_cache else None, 1 if graph else 0,
                           metrics_log.encode() if metrics_log else None,
                           1 if count_useful else 0, float(mlp_bound_cap), float(mlp_budget),
                           int(device_loop))
        self.log_capacity = int(log_capacity)
        self._ctx = C.c_void_p()
        st = lib().tc2_setup(probs, n, C.byref(opts), C.byref(self._ctx))
        if st != 0:
            raise TC2Error(st, "tc2_setup")

    def _results(self, res) -> List[Result]:
        out = []
        D = self.n_dir
        for r in res:
            x0 = _py_bsr(r.X0) if r.X0.row_ptr else None
            x1 = [_py_bsr(r.X1[d]) for d in range(D)] if r.X0.row_ptr else []
            out.append(Result(r.status, r.iters, r.branches.decode(), list(r.trace_x1h1[:D]),
                              r.tr_x0, r.idem_err, list(r.tr_x1[:D]), r.e0, list(r.e1[:D]),
                              r.emin, r.emax, r.seconds, r.useful_flops, r.executed_flops,
                              r.kept_blocks, r.screened_blocks, r.mlp_skipped_blocks,
                              r.ms_symbolic, r.ms_numeric, r.ms_compact,
                              r.numeric_launches, list(r.tile_shape), r.ms_tune,
                              list(r.useful_flops_kind), list(r.ms_numeric_kind),
                              list(r.numeric_launches_kind), r.graph_updates, x0, x1,
                              r.nominal_flops, r.union_flops, r.graph_captures,
                              r.mlp_updates, r.device_loop_updates))
        return out

    def run(self, stream: Optional[int] = None, check: bool = True) -> List[Result]:
        n = len(self.systems)
        res = (tc2_result * n)()
        st = lib().tc2_run(self._ctx, C.c_void_p(stream) if stream else None, res)
        if check and st < 0:
            raise TC2Error(st, "tc2_run")
        return self._results(res)

    def advance(self, max_updates: int, stream: Optional[int] = None):
        """Run at most ``max_updates`` updates (tc2_advance).  Returns
        (progress dict, results of the last solve finished in this call or
        None)."""
        n = len(self.systems)
        res = (tc2_result * n)()
        prog = tc2_progress()
        L = lib()
        L.tc2_advance.restype = C.c_int
        L.tc2_advance.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(tc2_progress),
                                  C.POINTER(tc2_result)]
        st = L.tc2_advance(self._ctx, C.c_void_p(stream) if stream else None, int(max_updates),
                           C.byref(prog), res)
        if st < 0:
            raise TC2Error(st, "tc2_advance")
        p = dict(updates=prog.updates, solves_completed=prog.solves_completed,
                 solve_open=bool(prog.solve_open), useful_flops=prog.useful_flops,
                 executed_flops=prog.executed_flops)
        return p, (self._results(res) if prog.solves_completed else None)

    def export_rows(self, system: int, rows: Sequence[int]):
        """Complete block rows of the current X0 and X1_d of one problem
        (tc2_export_rows): (X0, [X1_d]) as BSR with only those rows filled."""
        rr = np.ascontiguousarray(rows, dtype=np.int32)
        x0 = tc2_bsr()
        x1 = (tc2_bsr * 3)()
        L = lib()
        L.tc2_export_rows.restype = C.c_int
        L.tc2_export_rows.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(tc2_bsr), C.POINTER(tc2_bsr)]
        st = L.tc2_export_rows(self._ctx, int(system), rr.ctypes.data_as(C.POINTER(C.c_int32)),
                               len(rr), C.byref(x0), x1)
        if st != 0:
            raise TC2Error(st, "tc2_export_rows")
        try:
            return _py_bsr(x0), [_py_bsr(x1[d]) for d in range(self.n_dir)]
        finally:
            _release(x0)
            for d in range(self.n_dir):
                _release(x1[d])

    def iterate_size(self) -> int:
        n = C.c_int64()
        L = lib()
        L.tc2_iterate_size.restype = C.c_int
        L.tc2_iterate_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        st = L.tc2_iterate_size(self._ctx, C.byref(n))
        if st != 0:
            raise TC2Error(st, "tc2_iterate_size")
        return int(n.value)

    def export_entries(self, matrix: int, first: int, count: int, values: bool = True):
        """(rows, cols, vals) of entries [first, first + count) of the merged
        current iterate, matrix 0 = X0, 1 + d = X1_d (tc2_export_entries)."""
        b = self.systems[0].H.b
        rows = np.empty(max(count, 1), dtype=np.int32)
        cols = np.empty(max(count, 1), dtype=np.int32)
        vals = np.empty((max(count, 1), b, b), dtype=np.float64) if values else None
        L = lib()
        L.tc2_export_entries.restype = C.c_int
        L.tc2_export_entries.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double)]
        st = L.tc2_export_entries(self._ctx, int(matrix), int(first), int(count),
                                  rows.ctypes.data_as(C.POINTER(C.c_int32)),
                                  cols.ctypes.data_as(C.POINTER(C.c_int32)),
                                  vals.ctypes.data_as(C.POINTER(C.c_double)) if values else None)
        if st != 0:
            raise TC2Error(st, "tc2_export_entries")
        return rows[:count], cols[:count], (vals[:count] if values else None)

    def compare_entries(self, matrix: int, rows, cols, vals, detail: bool = False):
        """max |A - B| over the union of the patterns of the caller's entries A
        and matrix ``matrix`` of the current iterate B (tc2_compare_entries);
        with ``detail``, also a dict separating blocks both hold from blocks
        one side holds."""
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        out = C.c_double()
        det = (C.c_double * 6)()
        L = lib()
        L.tc2_compare_entries.restype = C.c_int
        L.tc2_compare_entries.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
        st = L.tc2_compare_entries(self._ctx, int(matrix), len(rows),
                                   rows.ctypes.data_as(C.POINTER(C.c_int32)),
                                   cols.ctypes.data_as(C.POINTER(C.c_int32)),
                                   vals.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out), det)
        if st != 0:
            raise TC2Error(st, "tc2_compare_entries")
        if not detail:
            return float(out.value)
        return float(out.value), dict(max_both=det[0], max_given_only=det[1],
                                      max_iterate_only=det[2], n_given_only=int(det[3]),
                                      n_iterate_only=int(det[4]), max_norm_one_side=det[5])

    def log(self, logits: bool = False):
        """(features n x 8, labels n) logged by the last run (1 = dropped,
        0 = kept, -1 = skipped by the network); with ``logits``, also the
        logits of the in-kernel network."""
        cap = self.log_capacity
        x = np.empty((max(cap, 1), MLP_IN), dtype=np.float32)
        y = np.empty(max(cap, 1), dtype=np.float32)
        z = np.empty(max(cap, 1), dtype=np.float32)
        L = lib()
        L.tc2_log_copy.restype = C.c_int64
        L.tc2_log_copy.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                   C.POINTER(C.c_float), C.c_int64]
        n = L.tc2_log_copy(self._ctx, _fptr(x), _fptr(y), _fptr(z), cap)
        if n < 0:
            raise TC2Error(int(n), "tc2_log_copy")
        if logits:
            return x[:n].copy(), y[:n].copy(), z[:n].copy()
        return x[:n].copy(), y[:n].copy()

    def close(self):
        if getattr(self, "_ctx", None):
            lib().tc2_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trim_memory(device: int = 0) -> None:
    """Return the library's pooled device memory (chunks kept for reuse by
    later buffers and contexts) to the driver (tc2_trim_memory)."""
    st = lib().tc2_trim_memory(int(device))
    if st != 0:
        raise TC2Error(st, "tc2_trim_memory")


def solve(systems, **kw) -> List[Result]:
    """One-shot setup + run + free."""
    s = Solver(systems, **kw)
    try:
        return s.run()
    finally:
        s.close()


def bsr_dense(m: BSR) -> np.ndarray:
    """Dense copy of a BSR result (for tests and checks)."""
    A = np.zeros((m.nb * m.b, m.nb * m.b))
    b = m.b
    for I in range(m.nb):
        for p in range(int(m.row_ptr[I]), int(m.row_ptr[I + 1])):
            J = int(m.col[p])
            A[I * b:(I + 1) * b, J * b:(J + 1) * b] = m.val[p]
    return A


# ---------------------------------------------------------------- dense O(N^3) path
DENSE_MAX_N = 40000


class tc2_dense_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("hip_stream", C.c_void_p),
                ("p0", C.POINTER(C.c_double)), ("p1", C.POINTER(C.c_double) * 3),
                ("eigenvalues", C.POINTER(C.c_double))]


class tc2_dense_result(C.Structure):
    _fields_ = [("status", C.c_int), ("e0", C.c_double), ("e1", C.c_double * 3),
                ("trace_p1h1", C.c_double * 3), ("tr_p0", C.c_double), ("gap", C.c_double),
                ("seconds", C.c_double), ("ms_eigh", C.c_double), ("ms_p0", C.c_double),
                ("ms_p1", C.c_double), ("flops_p1", C.c_double)]


@dataclass
class DenseResult:
    status: int
    e0: float
    e1: List[float]
    alpha: List[float]          # Tr(P1_d H1_d)
    tr_p0: float
    gap: float
    seconds: float
    ms_eigh: float
    ms_p0: float
    ms_p1: float
    flops_p1: float
    P0: Optional[np.ndarray] = None
    P1: List[np.ndarray] = field(default_factory=list)
    eigenvalues: Optional[np.ndarray] = None


def dense_response(system: System, export: bool = False, device: int = 0,
                   stream: Optional[int] = None) -> DenseResult:
    """P0, P1_d and their traces by diagonalisation (``tc2_dense_response``)."""
    keep: list = []
    p = tc2_problem()
    p.H = _c_bsr(system.H, keep)
    p.n_dir = len(system.H1)
    for d, h1 in enumerate(system.H1):
        p.H1[d] = _c_bsr(h1, keep)
    p.n_occ = int(system.n_occ)
    p.eps_drop, p.tol, p.max_iter = float(system.eps), float(system.tol), int(system.max_iter)
    N = system.H.nb * system.H.b
    D = len(system.H1)
    o = tc2_dense_options()
    o.device = int(device)
    o.hip_stream = C.c_void_p(stream) if stream else None
    P0 = P1 = ev = None
    if export:
        P0 = np.empty((N, N))
        P1 = [np.empty((N, N)) for _ in range(D)]
        ev = np.empty(N)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        o.p0 = dp(P0)
        for d in range(D):
            o.p1[d] = dp(P1[d])
        o.eigenvalues = dp(ev)
    r = tc2_dense_result()
    L = lib()
    L.tc2_dense_response.restype = C.c_int
    L.tc2_dense_response.argtypes = [C.POINTER(tc2_problem), C.POINTER(tc2_dense_options),
                                     C.POINTER(tc2_dense_result)]
    st = L.tc2_dense_response(C.byref(p), C.byref(o), C.byref(r))
    if st < 0:
        raise TC2Error(st, "tc2_dense_response")
    return DenseResult(r.status, r.e0, list(r.e1[:D]), list(r.trace_p1h1[:D]), r.tr_p0, r.gap,
                       r.seconds, r.ms_eigh, r.ms_p0, r.ms_p1, r.flops_p1, P0,
                       P1 if P1 is not None else [], ev)


# ---------------------------------------------------------------- Loewdin orthogonalisation
class tc2_lowdin_options(C.Structure):
    _fields_ = [("eps", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("device", C.c_int32), ("hip_stream", C.c_void_p)]


class tc2_lowdin_result(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int32), ("resid", C.c_double),
                ("lam", C.c_double), ("seconds", C.c_double), ("Z", tc2_bsr), ("H", tc2_bsr),
                ("H1", tc2_bsr * 3)]


@dataclass
class LowdinResult:
    status: int
    iters: int
    resid: float
    lam: float
    seconds: float
    Z: BSR                      # S^-1/2
    H: BSR                      # S^-1/2 H S^-1/2
    H1: List[BSR]               # S^-1/2 H1_d S^-1/2


def _release(m: tc2_bsr):
    L = lib()
    L.tc2_bsr_release.restype = None
    L.tc2_bsr_release.argtypes = [C.POINTER(tc2_bsr)]
    L.tc2_bsr_release(C.byref(m))


def lowdin(S: BSR, H: BSR, H1: Sequence[BSR] = (), eps: float = 1e-6, tol: float = 1e-9,
           max_iter: int = 50, device: int = 0, stream: Optional[int] = None) -> LowdinResult:
    """S^-1/2 by the Newton-Schulz iteration and the orthogonal forms of H and
    H1_d (``tc2_lowdin``)."""
    keep: list = []
    cS, cH = _c_bsr(S, keep), _c_bsr(H, keep)
    D = len(H1)
    arr = (tc2_bsr * 3)()
    for d, h in enumerate(H1):
        arr[d] = _c_bsr(h, keep)
    o = tc2_lowdin_options(float(eps), float(tol), int(max_iter), int(device),
                           C.c_void_p(stream) if stream else None)
    r = tc2_lowdin_result()
    L = lib()
    L.tc2_lowdin.restype = C.c_int
    L.tc2_lowdin.argtypes = [C.POINTER(tc2_bsr), C.POINTER(tc2_bsr), C.c_int32,
                             C.POINTER(tc2_bsr), C.POINTER(tc2_lowdin_options),
                             C.POINTER(tc2_lowdin_result)]
    st = L.tc2_lowdin(C.byref(cS), C.byref(cH), D, arr, C.byref(o), C.byref(r))
    if st < 0:
        raise TC2Error(st, "tc2_lowdin")
    try:
        out = LowdinResult(r.status, r.iters, r.resid, r.lam, r.seconds, _py_bsr(r.Z),
                           _py_bsr(r.H), [_py_bsr(r.H1[d]) for d in range(D)])
    finally:
        _release(r.Z)
        _release(r.H)
        for d in range(D):
            _release(r.H1[d])
    return out


def congruence(Z: BSR, X: BSR, eps: float = 1e-6, device: int = 0,
               stream: Optional[int] = None) -> BSR:
    """Z X Z with the block filter (``tc2_congruence``): the back-transform of
    a density matrix when Z = S^-1/2."""
    keep: list = []
    cZ, cX = _c_bsr(Z, keep), _c_bsr(X, keep)
    o = tc2_lowdin_options(float(eps), 1.0, 1, int(device), C.c_void_p(stream) if stream else None)
    out = tc2_bsr()
    sec = C.c_double()
    L = lib()
    L.tc2_congruence.restype = C.c_int
    L.tc2_congruence.argtypes = [C.POINTER(tc2_bsr), C.POINTER(tc2_bsr),
                                 C.POINTER(tc2_lowdin_options), C.POINTER(tc2_bsr),
                                 C.POINTER(C.c_double)]
    st = L.tc2_congruence(C.byref(cZ), C.byref(cX), C.byref(o), C.byref(out), C.byref(sec))
    if st < 0:
        raise TC2Error(st, "tc2_congruence")
    try:
        return _py_bsr(out)
    finally:
        _release(out)


# ---------------------------------------------------------------- moving overlap (displacements)
class tc2_lowdin_response_result(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int32), ("resid", C.c_double),
                ("lam", C.c_double), ("seconds", C.c_double), ("Z", tc2_bsr), ("H", tc2_bsr),
                ("Z1", tc2_bsr * 3), ("H1", tc2_bsr * 3)]


@dataclass
class LowdinResponseResult:
    status: int
    iters: int
    resid: float
    lam: float
    seconds: float
    Z: BSR                      # S^-1/2
    H: BSR                      # S^-1/2 H S^-1/2
    Z1: List[BSR]               # derivative of S^-1/2 along S1_d
    H1: List[BSR]               # Z1 H Z + Z H1_d Z + Z H Z1


def lowdin_response(S: BSR, H: BSR, H1: Sequence[BSR], S1: Sequence[BSR], eps: float = 1e-6,
                    tol: float = 1e-9, max_iter: int = 50, device: int = 0,
                    stream: Optional[int] = None) -> LowdinResponseResult:
    """S^-1/2, its derivatives along S1_d, and the orthogonal forms of H and of
    perturbations that move the overlap (``tc2_lowdin_response``)."""
    keep: list = []
    cS, cH = _c_bsr(S, keep), _c_bsr(H, keep)
    D = len(H1)
    assert len(S1) == D
    a1, s1 = (tc2_bsr * 3)(), (tc2_bsr * 3)()
    for d in range(D):
        a1[d] = _c_bsr(H1[d], keep)
        s1[d] = _c_bsr(S1[d], keep)
    o = tc2_lowdin_options(float(eps), float(tol), int(max_iter), int(device),
                           C.c_void_p(stream) if stream else None)
    r = tc2_lowdin_response_result()
    L = lib()
    L.tc2_lowdin_response.restype = C.c_int
    L.tc2_lowdin_response.argtypes = [C.POINTER(tc2_bsr), C.POINTER(tc2_bsr), C.c_int32,
                                      C.POINTER(tc2_bsr), C.POINTER(tc2_bsr),
                                      C.POINTER(tc2_lowdin_options),
                                      C.POINTER(tc2_lowdin_response_result)]
    st = L.tc2_lowdin_response(C.byref(cS), C.byref(cH), D, a1, s1, C.byref(o), C.byref(r))
    if st < 0:
        raise TC2Error(st, "tc2_lowdin_response")
    try:
        out = LowdinResponseResult(r.status, r.iters, r.resid, r.lam, r.seconds, _py_bsr(r.Z),
                                   _py_bsr(r.H), [_py_bsr(r.Z1[d]) for d in range(D)],
                                   [_py_bsr(r.H1[d]) for d in range(D)])
    finally:
        _release(r.Z)
        _release(r.H)
        for d in range(D):
            _release(r.Z1[d])
            _release(r.H1[d])
    return out


def congruence_response(Z: BSR, Z1: BSR, X: BSR, X1: BSR, eps: float = 1e-6, device: int = 0,
                        stream: Optional[int] = None) -> BSR:
    """Z1 X Z + Z X1 Z + Z X Z1 (``tc2_congruence_response``)."""
    keep: list = []
    cZ, cZ1, cX, cX1 = (_c_bsr(m, keep) for m in (Z, Z1, X, X1))
    o = tc2_lowdin_options(float(eps), 1.0, 1, int(device), C.c_void_p(stream) if stream else None)
    out = tc2_bsr()
    sec = C.c_double()
    L = lib()
    L.tc2_congruence_response.restype = C.c_int
    L.tc2_congruence_response.argtypes = [C.POINTER(tc2_bsr)] * 4 + [
        C.POINTER(tc2_lowdin_options), C.POINTER(tc2_bsr), C.POINTER(C.c_double)]
    st = L.tc2_congruence_response(C.byref(cZ), C.byref(cZ1), C.byref(cX), C.byref(cX1),
                                   C.byref(o), C.byref(out), C.byref(sec))
    if st < 0:
        raise TC2Error(st, "tc2_congruence_response")
    try:
        return _py_bsr(out)
    finally:
        _release(out)
