"""Closed-form limits of TC2 and TC2-CPSCF (test infrastructure).

Without truncation the TC2 iterates converge to the projector onto the
N_occ lowest eigenvectors of H (Sec. 2.2: the density matrix as a sum over
occupied states) and the response iterates to its derivative, which the
O(N^3) route of Sec. 2.1 writes with the expansion C1 = C0 U1,
U1_pq = -(C0^T H1 C0)_pq / (e_p - e_q), U1_pp = 0 (Eq. cpscf-LCAO), and
P1 = sum_i f_i (C1_i C0_i^T + C0_i C1_i^T) with f_i = 1 in the orthonormal,
spin-free notation used by TC2.
"""
from __future__ import annotations

import numpy as np


def _eig(H):
    e, C = np.linalg.eigh(np.asarray(H, dtype=np.float64))
    return e, C


def exact_projector(H, n_occ: int) -> np.ndarray:
    """P0 = sum_{i <= N_occ} c_i c_i^T from a dense diagonalisation."""
    e, C = _eig(H)
    Co = C[:, :n_occ]
    return Co @ Co.T


def exact_response(H, H1, n_occ: int) -> np.ndarray:
    """P1 through the sum over states: only occupied-virtual pairs survive
    because U1_pp = 0 and the occupied-occupied terms cancel in P1."""
    e, C = _eig(H)
    Co, Cv = C[:, :n_occ], C[:, n_occ:]
    eo, ev = e[:n_occ], e[n_occ:]
    # C1_i = sum_a C_a U_ai with U_ai = -(C^T H1 C)_ai / (e_a - e_i)
    #      = (C^T H1 C)_ai / (e_i - e_a)
    M = (Co.T @ H1 @ Cv) / (eo[:, None] - ev[None, :])      # (occ, virt)
    T = Co @ M @ Cv.T                                       # sum_i c_i C1_i^T
    return T + T.T


def exact_alpha(H, H1, n_occ: int) -> float:
    """Tr(P1 H1) = 2 sum_{i occ, a virt} |<i|H1|a>|^2 / (e_i - e_a)."""
    e, C = _eig(H)
    Co, Cv = C[:, :n_occ], C[:, n_occ:]
    eo, ev = e[:n_occ], e[n_occ:]
    V = Co.T @ H1 @ Cv
    return float(2.0 * np.sum(V * V / (eo[:, None] - ev[None, :])))
