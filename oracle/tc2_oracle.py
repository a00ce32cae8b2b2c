"""Dense FP64 oracle for the TC2 recursion and its response (test infrastructure).

Plain, slow and literal: every matrix is dense, every product is a numpy
matmul, every step follows the paper (Shang et al., "Efficient parallel
linear scaling method to get the response density matrix in all-electron
real-space DFPT", Sec. 2.2 "The O(N) method to get the first order density
matrix").  Nothing here is blocked, fused or reordered beyond what the paper
states.  The GPU library shares no code with this file.

Readings of points the paper leaves open (they are the same for the GPU
library, which implements them independently):

* spectral bounds: Gershgorin discs of the scalar rows of the full H, FP64;
* branch: SQUARE when Tr X0 >= N_occ (ties go to SQUARE); the response
  uses the same branch as X0;
* filter ("NTPoly-filter", Sec. 2.3): applied after each update, per atom
  block, by Frobenius norm: an off-diagonal block (I, J), I < J, whose norm is
  strictly below ``eps`` is zeroed together with its mirror (J, I); each of
  X0 and X1_d is filtered on its own; diagonal blocks are never filtered;
  the initial matrices are not filtered;
* stopping ("NTPoly-tolerance", Sec. 2.3; band energies of Sec. 2.2):
  after k >= 2 updates, stop when the change of E0 = Tr(X0 H), of every
  E1_d = Tr(X1_d H) and of every alpha_d = Tr(X1_d H1_d) is below ``tol``;
* stall guard: once |iota| < 1, with iota = Tr X0 - ||X0||_F^2, stop when
  |iota_k| >= |iota_{k-2}| (precision floor reached);
* optional closing pair: two further steps, the first by the trace rule, the
  second with the opposite branch.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SQUARE = 1
DOUBLE = 0

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_FLOOR = 2


def bsr_to_dense(nb: int, b: int, row_ptr, col, val) -> np.ndarray:
    """Scatter a block-sparse matrix (row pointer, column index, b x b
    row-major blocks) into a dense FP64 array."""
    A = np.zeros((nb * b, nb * b))
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    val = np.asarray(val, dtype=np.float64).reshape(-1, b, b)
    for I in range(nb):
        for p in range(int(row_ptr[I]), int(row_ptr[I + 1])):
            J = int(col[p])
            A[I * b:(I + 1) * b, J * b:(J + 1) * b] = val[p]
    return A


def gershgorin(H: np.ndarray):
    """Spectral bounds of H by Gershgorin's circle theorem (Sec. 2.2, used for
    the TC2 initial guess): each eigenvalue lies in some disc centred at
    H_ii with radius sum_{j != i} |H_ij|."""
    d = np.diag(H)
    radius = np.abs(H).sum(axis=1) - np.abs(d)
    return float(np.min(d - radius)), float(np.max(d + radius))


def tc2_init(H: np.ndarray, H1s: Sequence[np.ndarray], emin: float, emax: float):
    """Initial matrices of the TC2 recursion and of its response (Sec. 2.2):
    X0 = (emax*I - H) / (emax - emin) and X1 = -H1 / (emax - emin)."""
    W = emax - emin
    n = H.shape[0]
    X0 = (emax * np.eye(n) - H) / W
    X1s = [-H1 / W for H1 in H1s]
    return X0, X1s


def block_drop(X: np.ndarray, b: int, eps: float) -> np.ndarray:
    """Filter of small matrix elements, made block-wise: zero every
    off-diagonal b x b block pair (I, J), (J, I) whose upper block (I < J) has
    Frobenius norm strictly below eps.  Returns a new array."""
    if eps <= 0.0:
        return X.copy()
    nb = X.shape[0] // b
    Y = X.copy()
    blocks = X.reshape(nb, b, nb, b)
    norms = np.sqrt(np.einsum("iajb,iajb->ij", blocks, blocks))
    I, J = np.nonzero(np.triu(norms < eps, k=1))
    for i, j in zip(I, J):
        Y[i * b:(i + 1) * b, j * b:(j + 1) * b] = 0.0
        Y[j * b:(j + 1) * b, i * b:(i + 1) * b] = 0.0
    return Y


def tc2_step(X0: np.ndarray, X1s: Sequence[np.ndarray], square: bool):
    """One TC2 update (Eq. TC2) and one TC2-CPSCF update (Eq. TC2-CPSCF),
    both with the branch chosen from Tr X0 of the current iterate:
    SQUARE:  X0 <- X0 X0,          X1 <- X1 X0 + X0 X1;
    DOUBLE:  X0 <- 2 X0 - X0 X0,   X1 <- 2 X1 - X1 X0 - X0 X1."""
    X2 = X0 @ X0
    S = [X1 @ X0 + X0 @ X1 for X1 in X1s]
    if square:
        return X2, S
    return 2.0 * X0 - X2, [2.0 * X1 - s for X1, s in zip(X1s, S)]


def band_energies(X0, X1s, H, H1s):
    """E0 = Tr(X0 H) and E1_d = Tr(X1_d H) (band energies of Sec. 2.2), and
    alpha_d = Tr(X1_d H1_d), the raw polarizability trace."""
    E0 = float(np.sum(X0 * H.T))
    E1 = [float(np.sum(X1 * H.T)) for X1 in X1s]
    al = [float(np.sum(X1 * H1.T)) for X1, H1 in zip(X1s, H1s)]
    return E0, E1, al


def block_nonzero(X: np.ndarray, b: int) -> np.ndarray:
    """(nb x nb) flags: block (I, J) of X has a nonzero element."""
    nb = X.shape[0] // b
    return np.any(X.reshape(nb, b, nb, b) != 0.0, axis=(1, 3))


def useful_products(prev: Sequence[np.ndarray], new: Sequence[np.ndarray], b: int) -> int:
    """Useful block products of one update, from the iterate before it (prev =
    [X0, X1_1, ..]) and after it (new, filtered).  The work of an update of
    Eq. TC2 / TC2-CPSCF counted on stored blocks only, over the upper
    triangle of the output (the lower half is its mirror):

    * X0 X0: triples (I, K, J), I <= J, with X0_IK and X0_KJ nonzero and the
      new X0_IJ nonzero (kept by the filter);
    * X0 X1_d + X1_d X0: triples with X0_IK and X1_d,KJ nonzero, plus triples
      with X1_d,IK and X0_KJ nonzero, on outputs where the new X1_d,IJ is
      nonzero.

    Each product is 2 b^3 flops."""
    M = [block_nonzero(X, b).astype(np.int64) for X in prev]
    N = [block_nonzero(X, b) for X in new]
    up = np.triu(np.ones(N[0].shape, dtype=bool))
    total = int(((M[0] @ M[0]) * (N[0] & up)).sum())
    for d in range(1, len(prev)):
        total += int(((M[0] @ M[d] + M[d] @ M[0]) * (N[d] & up)).sum())
    return total


def stopping_rule(k: int, prev, cur, iotas: Sequence[float], tol: float,
                  stall_guard: bool = True) -> Optional[int]:
    """Stopping decision after update k (k = 1, 2, ...), from the scalars of
    the previous and the current iterate.

    ``prev`` and ``cur`` are (E0, [E1_d], [alpha_d]) as returned by
    band_energies; ``iotas`` holds iota_1 .. iota_k, iota = Tr X0 - ||X0||_F^2.

    * Convergence (tolerance test of Sec. 2.3 on the band energies of
      Sec. 2.2): k >= 2 and every one of |dE0|, |dE1_d|, |d alpha_d| is below
      tol -> STATUS_OK.  alpha_d takes part because E1_d = Tr(X1_d H) tends to
      0 for every response, converged or not.
    * Stall guard (precision floor of the recursion in finite precision):
      k >= 3, |iota_k| < 1 and |iota_k| >= |iota_{k-2}| -> STATUS_FLOOR.  The
      comparison skips one update because the two branches alternate near the
      fixed point and iota falls over pairs of updates, not every update.
    * Otherwise None (continue)."""
    d = [abs(cur[0] - prev[0])]
    d += [abs(a - c) for a, c in zip(cur[1], prev[1])]
    d += [abs(a - c) for a, c in zip(cur[2], prev[2])]
    if k >= 2 and max(d) < tol:
        return STATUS_OK
    if stall_guard and k >= 3 and abs(iotas[k - 1]) < 1.0 and \
            abs(iotas[k - 1]) >= abs(iotas[k - 3]):
        return STATUS_FLOOR
    return None


@dataclass
class OracleResult:
    X0: np.ndarray
    X1: List[np.ndarray]
    alpha: List[float]
    iters: int
    branches: str                  # 'S' (square) / 'D' (double) per update
    status: int
    emin: float
    emax: float
    history: List[dict] = field(default_factory=list)

    @property
    def tr_x0(self) -> float:
        return float(np.trace(self.X0))


def tc2_solve(H: np.ndarray, H1s: Sequence[np.ndarray], n_occ: int, b: int,
              eps: float, tol: float, max_iter: int = 100,
              replay: Optional[str] = None, closing_pair: bool = False,
              stall_guard: bool = True, keep_history: bool = False) -> OracleResult:
    """TC2 purification of X0 coupled with its response X1 (Sec. 2.2), in
    dense FP64, with the block filter and the band-energy stopping test.

    ``replay`` forces the branch of every update ('S'/'D' per step) and runs
    exactly len(replay) updates; ``closing_pair`` appends the two closing
    steps (trace rule, then the opposite branch)."""
    H = np.asarray(H, dtype=np.float64)
    H1s = [np.asarray(h, dtype=np.float64) for h in H1s]
    n = H.shape[0]
    emin, emax = gershgorin(H)
    if n_occ == 0 or n_occ == n:
        X0 = np.zeros((n, n)) if n_occ == 0 else np.eye(n)
        return OracleResult(X0, [np.zeros((n, n)) for _ in H1s],
                            [0.0] * len(H1s), 0, "", STATUS_OK, emin, emax)
    X0, X1s = tc2_init(H, H1s, emin, emax)
    prev = band_energies(X0, X1s, H, H1s)
    iotas: List[float] = []
    branches = []
    history = []
    status = STATUS_NOT_CONVERGED
    steps = len(replay) if replay is not None else max_iter
    for k in range(1, steps + 1):
        if replay is not None:
            square = replay[k - 1] == "S"
        else:
            square = np.trace(X0) >= n_occ
        branches.append("S" if square else "D")
        X0, X1s = tc2_step(X0, X1s, square)
        X0 = block_drop(X0, b, eps)
        X1s = [block_drop(X1, b, eps) for X1 in X1s]
        cur = band_energies(X0, X1s, H, H1s)
        iota = float(np.trace(X0) - np.sum(X0 * X0))
        iotas.append(iota)
        if keep_history:
            history.append(dict(k=k, branch=branches[-1], tr=float(np.trace(X0)),
                                E0=cur[0], E1=list(cur[1]), alpha=list(cur[2]),
                                iota=iota))
        if replay is None:
            stop = stopping_rule(k, prev, cur, iotas, tol, stall_guard)
            if stop is not None:
                status = stop
                prev = cur
                break
        prev = cur
    else:
        if replay is not None:
            status = STATUS_OK
    if closing_pair:
        first = np.trace(X0) >= n_occ
        for square in (first, not first):
            branches.append("S" if square else "D")
            X0, X1s = tc2_step(X0, X1s, square)
            X0 = block_drop(X0, b, eps)
            X1s = [block_drop(X1, b, eps) for X1 in X1s]
        prev = band_energies(X0, X1s, H, H1s)
    return OracleResult(X0, X1s, list(prev[2]), len(branches), "".join(branches),
                        status, emin, emax, history)


def solve_system(sys, replay: Optional[str] = None, closing_pair: bool = False,
                 eps: Optional[float] = None, tol: Optional[float] = None,
                 max_iter: Optional[int] = None, keep_history: bool = False,
                 stall_guard: bool = True) -> OracleResult:
    """Convenience wrapper taking a generated system (BSR H, H1, n_occ)."""
    H = bsr_to_dense(sys.H.nb, sys.H.b, sys.H.row_ptr, sys.H.col, sys.H.val)
    H1s = [bsr_to_dense(h.nb, h.b, h.row_ptr, h.col, h.val) for h in sys.H1]
    return tc2_solve(H, H1s, sys.n_occ, sys.H.b,
                     sys.eps if eps is None else eps,
                     sys.tol if tol is None else tol,
                     sys.max_iter if max_iter is None else max_iter,
                     replay=replay, closing_pair=closing_pair,
                     keep_history=keep_history, stall_guard=stall_guard)
