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
  mirror them, so that the result is exactly symmetric.  Without the filter
  these products are symmetric up to rounding; with it, Z and Y are only
  approximately functions of S and the computed product is symmetric up to
  what the filter removed.  The part the mirror discards is pinned below
  eps per element (per product and on the final S^-1/2, against the plain
  product of every step: ``mirror=False``).  The inner product of
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
                           max_iter: int, mirror: bool = True) -> InvSqrt:
    """S^-1/2 by the coupled Newton-Schulz iteration with the block filter.

    ``mirror=False`` forms every product plainly (``product``: each block of
    the computed product filtered on its own, nothing mirrored).  Under the
    filter Z and Y are no longer exact functions of S, so Z Y is symmetric
    only up to what the filter removed; the tests bound the difference
    between the two readings by eps."""
    sym = symmetric_product if mirror else product
    N = S.shape[0]
    lam = gershgorin_upper(S)
    Y = S / lam
    Z = np.eye(N)
    iters = 0
    prev = None
    while True:
        M = sym(Z, Y, b, eps)
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
        Y = sym(Y, T, b, eps)
        Z = sym(Z, T, b, eps)
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


# ---------------------------------------------------------------- perturbed overlap
# An atomic displacement moves basis functions, so the overlap changes too
# (S1 != 0) and the response of the orthogonal form gains the derivative Z1 of
# S^-1/2 (the non-orthogonal response the paper names as the next use of the
# formalism).  Z1 comes from differentiating every step of the same
# Newton-Schulz iteration; the orthogonal perturbation and the back-transform
# follow by the product rule:
#     H1_orth = Z1 H Z + Z H1 Z + Z H Z1,   P1 = Z1 X0 Z + Z X1 Z + Z X0 Z1.
# Each derivative is a sum of two products, filtered after the sum; where the
# sum is symmetric (M1, Y1, Z1, H1_orth, P1) its upper blocks are mirrored.


def symmetric_product2(A, B, A2, B2, b: int, eps: float) -> np.ndarray:
    """A B + A2 B2 for a sum known to be symmetric: upper blocks mirrored,
    then the block filter."""
    return symmetric_product(np.hstack([A, A2]), np.vstack([B, B2]), b, eps)


def product2(A, B, A2, B2, b: int, eps: float) -> np.ndarray:
    """A B + A2 B2, each off-diagonal block filtered on its own."""
    return product(np.hstack([A, A2]), np.vstack([B, B2]), b, eps)


@dataclass
class InvSqrtResponse:
    Z: np.ndarray               # S^-1/2
    Z1: List[np.ndarray]        # d S^-1/2 for each S1_d
    iters: int
    resid: float
    lam: float
    status: int


def newton_schulz_response(S: np.ndarray, S1s: Sequence[np.ndarray], b: int, eps: float,
                           tol: float, max_iter: int) -> InvSqrtResponse:
    """The coupled Newton-Schulz iteration of newton_schulz_inv_sqrt together
    with its derivative along each S1_d (same updates, same stopping tests on
    the unperturbed residual)."""
    N = S.shape[0]
    lam = gershgorin_upper(S)
    Y, Z = S / lam, np.eye(N)
    Y1 = [s1 / lam for s1 in S1s]
    Z1 = [np.zeros((N, N)) for _ in S1s]
    iters, prev = 0, None
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
        T1 = [-0.5 * symmetric_product2(z1, Y, Z, y1, b, eps) for z1, y1 in zip(Z1, Y1)]
        Y1 = [symmetric_product2(y1, T, Y, t1, b, eps) for y1, t1 in zip(Y1, T1)]
        Z1 = [symmetric_product2(z1, T, Z, t1, b, eps) for z1, t1 in zip(Z1, T1)]
        Y = symmetric_product(Y, T, b, eps)
        Z = symmetric_product(Z, T, b, eps)
        iters += 1
    return InvSqrtResponse(Z / np.sqrt(lam), [z1 / np.sqrt(lam) for z1 in Z1], iters, resid,
                           lam, status)


def congruence_response(Z, Z1, X, X1, b: int, eps: float) -> np.ndarray:
    """Z1 X Z + Z X1 Z + Z X Z1 as (Z1 X + Z X1) Z + (Z X) Z1."""
    Q1 = product2(Z1, X, Z, X1, b, eps)
    Q = product(Z, X, b, eps)
    return symmetric_product2(Q1, Z, Q, Z1, b, eps)


@dataclass
class LowdinResponse:
    Z: np.ndarray
    Z1: List[np.ndarray]
    H: np.ndarray
    H1: List[np.ndarray]        # H1_orth_d = Z1 H Z + Z H1_d Z + Z H Z1
    iters: int
    resid: float
    lam: float
    status: int


def lowdin_response(S, S1s, H, H1s, b: int, eps: float, tol: float,
                    max_iter: int) -> LowdinResponse:
    """Orthogonal forms for perturbations that change both H (H1_d) and S
    (S1_d)."""
    r = newton_schulz_response(S, S1s, b, eps, tol, max_iter)
    Ho = congruence(r.Z, H, b, eps)
    H1o = [congruence_response(r.Z, z1, H, h1, b, eps) for z1, h1 in zip(r.Z1, H1s)]
    return LowdinResponse(r.Z, r.Z1, Ho, H1o, r.iters, r.resid, r.lam, r.status)

