"""Dense FP64 oracle of the Loewdin orthogonalisation (test infrastructure).

Sec. 2.2 brings a non-orthogonal problem (H, S) to the orthogonal form
H_orth = S^-1/2 H S^-1/2 before the TC2 cycles, and transforms the converged
P0_orth and P1_orth back with P = S^-1/2 P_orth S^-1/2.  S^-1/2 comes from a
linear-scaling Newton-Schulz iteration.  This module takes those steps on
dense matrices, with the block filter of Sec. 2.3 applied after every
product.  Nothing here is blocked, fused or reordered; the GPU library shares
no code with it.

Readings of points the paper leaves open (the GPU library implements the
same readings on its own):

* Newton-Schulz form: the coupled iteration for the inverse square root
  (Higham's stable form of the iteration the paper cites), started from
  Y0 = S / lam and Z0 = I, with lam the Gershgorin upper bound of S so that
  the spectrum of Y0 lies in (0, 1]:
      M = Z Y,  T = (3 I - M) / 2,  Y <- Y T,  Z <- Z T,
  which takes Y to (S/lam)^1/2 and Z to (S/lam)^-1/2; then S^-1/2 = Z / sqrt(lam).
* Stopping: before each update, stop when ||Z Y - I||_F / sqrt(N) < tol; at
  most max_iter updates.  Stall guard (as for TC2, a precision floor): after
  an update, stop when that residual fell by less than half, because the
  filter or rounding, not the iteration, then sets it.
* Products whose exact value is symmetric (Z Y, Y T, Z T, and the outer
  product of a congruence) keep the upper blocks of the computed product and
  mirror them, so that the result is exactly symmetric.  The inner product of
  a congruence, Q = Z X, is not symmetric and is kept whole.
* Filter: after every product, an off-diagonal block whose Frobenius norm is
  strictly below eps is zeroed (for a symmetric product, with its mirror).
  The initial Y0 and Z0 and the scaled result are not filtered.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from .tc2_oracle import block_drop

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_FLOOR = 2


def gershgorin_upper(S: np.ndarray) -> float:
    """Upper end of the union of the Gershgorin discs of the scalar rows."""
    d = np.diag(S)
    r = np.abs(S).sum(axis=1) - np.abs(d)
    return float(np.max(d + r))


def symmetric_product(A: np.ndarray, B: np.ndarray, b: int, eps: float) -> np.ndarray:
    """A B for a product known to be symmetric: upper blocks mirrored, then
    the block filter."""
    C = A @ B
    nb = C.shape[0] // b
    mask = np.kron(np.triu(np.ones((nb, nb))), np.ones((b, b))).astype(bool)
    U = np.where(mask, C, 0.0)
    Cs = U + U.T - np.diag(np.diag(U))
    # the diagonal blocks: their upper scalar triangle mirrored as well
    for I in range(nb):
        blk = C[I * b:(I + 1) * b, I * b:(I + 1) * b]
        t = np.triu(blk)
        Cs[I * b:(I + 1) * b, I * b:(I + 1) * b] = t + t.T - np.diag(np.diag(t))
    return block_drop(Cs, b, eps)


def product(A: np.ndarray, B: np.ndarray, b: int, eps: float) -> np.ndarray:
    """A B with the block filter applied to every off-diagonal block on its
    own (the result need not be symmetric)."""
    C = A @ B
    if eps <= 0.0:
        return C
    nb = C.shape[0] // b
    blocks = C.reshape(nb, b, nb, b)
    norms = np.sqrt(np.einsum("iajb,iajb->ij", blocks, blocks))
    keep = (norms >= eps) | np.eye(nb, dtype=bool)
    return C * np.kron(keep, np.ones((b, b)))


@dataclass
class InvSqrt:
    Z: np.ndarray          # S^-1/2
    iters: int             # updates performed
    resid: float           # ||Z Y - I||_F / sqrt(N) at the last test
    lam: float             # scale of S
    status: int


def newton_schulz_inv_sqrt(S: np.ndarray, b: int, eps: float, tol: float,
                           max_iter: int) -> InvSqrt:
    """S^-1/2 by the coupled Newton-Schulz iteration with the block filter."""
    N = S.shape[0]
    lam = gershgorin_upper(S)
    Y = S / lam
    Z = np.eye(N)
    iters = 0
    prev = None
    while True:
        M = symmetric_product(Z, Y, b, eps)
        resid = float(np.linalg.norm(M - np.eye(N)) / np.sqrt(N))
        if resid < tol:
            status = STATUS_OK
            break
        if prev is not None and resid > 0.5 * prev:
            status = STATUS_FLOOR
            break
        prev = resid
        if iters == max_iter:
            status = STATUS_NOT_CONVERGED
            break
        T = 0.5 * (3.0 * np.eye(N) - M)
        Y = symmetric_product(Y, T, b, eps)
        Z = symmetric_product(Z, T, b, eps)
        iters += 1
    return InvSqrt(Z / np.sqrt(lam), iters, resid, lam, status)


def congruence(Z: np.ndarray, X: np.ndarray, b: int, eps: float) -> np.ndarray:
    """Z X Z as two filtered products: Q = Z X (kept whole), then Q Z
    (symmetric: upper blocks mirrored)."""
    return symmetric_product(product(Z, X, b, eps), Z, b, eps)


@dataclass
class Lowdin:
    Z: np.ndarray
    H: np.ndarray
    H1: List[np.ndarray]
    iters: int
    resid: float
    lam: float
    status: int


def lowdin(S: np.ndarray, H: np.ndarray, H1s: Sequence[np.ndarray], b: int, eps: float,
           tol: float, max_iter: int) -> Lowdin:
    """Orthogonal forms H_orth = Z H Z and H1_orth = Z H1 Z with Z = S^-1/2
    (Sec. 2.2)."""
    r = newton_schulz_inv_sqrt(S, b, eps, tol, max_iter)
    Ho = congruence(r.Z, H, b, eps)
    H1o = [congruence(r.Z, h, b, eps) for h in H1s]
    return Lowdin(r.Z, Ho, H1o, r.iters, r.resid, r.lam, r.status)
