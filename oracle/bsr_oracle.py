"""Block-list FP64 oracle of the first TC2 / TC2-CPSCF updates for systems too
large for dense matrices (test infrastructure).

The dense oracle (tc2_oracle) stops at N ~ 13000.  This module takes the same
arithmetic to block lists, so that full-size systems (N = 104000 and 351000)
can be checked on sampled block rows.  Nothing here is shared with the GPU
library; only the tests and the CPU-baseline leg of the benchmark use it.

What one update computes (Sec. 2.2, Eq. TC2 and Eq. TC2-CPSCF; filter of
Sec. 2.3 made block-wise, as in the dense oracle):

    SQUARE:  X0' = X0 X0,          X1_d' = X0 X1_d + X1_d X0
    DOUBLE:  X0' = 2X0 - X0 X0,    X1_d' = 2X1_d - (X0 X1_d + X1_d X0)

then every off-diagonal block of each matrix whose Frobenius norm is below
eps is zeroed (diagonal blocks never).

Block form.  All matrices are symmetric, so X_KJ = X_JK^T and one output
block is a sum over the block columns common to rows I and J:

    (X0 X0)_IJ           = sum_K X0_IK X0_JK^T
    (X0 X1 + X1 X0)_IJ   = sum_K (X0_IK X1_JK^T + X1_IK X0_JK^T)

Rows of an update are formed by Gustavson's row-wise product (Algorithm 1
of Sec. 2.3): row I of X X is the sum over K in row I of X_IK times row K,
so the candidate columns J of row I are the union of the columns of those
rows K.  Diagonal blocks alone (for traces) use the block form
(X X)_II = sum_K X_IK X_IK^T.

Computing row I of X_k needs row I and the rows K of row I of X_{k-1}, so
sampled rows of a later update need the rows of the earlier updates within
a ball of the coupling graph (the 'cone').  Branches come
from Tr X_k, which needs only the diagonal blocks of X_k: the diagonal
blocks of every row of X_k need the complete rows of X_{k-1}.

An iterate is a dict {I: (cols, vals)}: cols an int array sorted ascending,
vals an array (len(cols), 1 + D, b, b) holding X0 and X1_1 .. X1_D of the
union pattern (a matrix that dropped a block stores zeros there).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

Rows = Dict[int, Tuple[np.ndarray, np.ndarray]]

# b x b block products performed so far (for timing the oracle: its rate is
# this count times 2 b^3 over the elapsed time)
PRODUCTS = [0]


def gershgorin_rows(H) -> Tuple[float, float]:
    """Gershgorin bounds of a BSR H (row_ptr, col, val with b x b row-major
    blocks): every eigenvalue lies in a disc centred at H_ii with radius
    sum_{j != i} |H_ij| over the scalar row i (Sec. 2.2)."""
    b = H.b
    lo, hi = np.inf, -np.inf
    for I in range(H.nb):
        p0, p1 = int(H.row_ptr[I]), int(H.row_ptr[I + 1])
        blocks = np.asarray(H.val[p0:p1]).reshape(-1, b, b)
        absrow = np.abs(blocks).sum(axis=(0, 2))           # sum_j |H_ij| over the block row
        d = None
        for q, J in enumerate(H.col[p0:p1]):
            if J == I:
                d = np.diag(blocks[q])
        rad = absrow - np.abs(d)
        lo = min(lo, float(np.min(d - rad)))
        hi = max(hi, float(np.max(d + rad)))
    return lo, hi


def init_rows(H, H1s: Sequence, emin: float, emax: float, rows: Optional[Iterable[int]] = None) -> Rows:
    """X0 = (emax I - H)/W and X1_d = -H1_d/W (Sec. 2.2), W = emax - emin, on the
    union of the patterns of H and the H1_d; no filter at init."""
    W = emax - emin
    b, D = H.b, len(H1s)
    out: Rows = {}
    for I in (range(H.nb) if rows is None else rows):
        blocks = {}
        def put(m, J, v):
            blocks.setdefault(int(J), np.zeros((1 + D, b, b)))[m] = v
        for p in range(int(H.row_ptr[I]), int(H.row_ptr[I + 1])):
            J = int(H.col[p])
            v = -np.asarray(H.val[p]).reshape(b, b) / W
            if J == I:
                v = v + np.eye(b) * (emax / W)
            put(0, J, v)
        for d, H1 in enumerate(H1s):
            for p in range(int(H1.row_ptr[I]), int(H1.row_ptr[I + 1])):
                put(1 + d, H1.col[p], -np.asarray(H1.val[p]).reshape(b, b) / W)
        cols = np.array(sorted(blocks), dtype=np.int64)
        out[I] = (cols, np.stack([blocks[J] for J in cols]))
    return out


def upper_block(X: Rows, I: int, J: int) -> np.ndarray:
    """(X0 X0)_IJ and (X0 X1_d + X1_d X0)_IJ for I <= J, as an array
    (1 + D, b, b), summed over the common block columns K of rows I and J."""
    ci, vi = X[I]
    cj, vj = X[J]
    _, a, c = np.intersect1d(ci, cj, assume_unique=True, return_indices=True)
    A, B = vi[a], vj[c]                                    # (nK, 1 + D, b, b)
    D = vi.shape[1] - 1
    out = np.zeros(vi.shape[1:])
    PRODUCTS[0] += len(a) * (1 + 2 * (vi.shape[1] - 1))
    if len(a) == 0:
        return out
    BT = np.swapaxes(B, -1, -2)                            # X_KJ = X_JK^T
    out[0] = np.matmul(A[:, 0], BT[:, 0]).sum(axis=0)
    for d in range(D):
        out[1 + d] = (np.matmul(A[:, 0], BT[:, 1 + d]) + np.matmul(A[:, 1 + d], BT[:, 0])).sum(axis=0)
    return out


def combine_and_filter(C: np.ndarray, old: Optional[np.ndarray], square: bool, eps: float,
                       diag: bool) -> np.ndarray:
    """The branch of Eq. TC2 / TC2-CPSCF applied to one block (C holds the
    products, old the block of the previous iterate or None when absent),
    then the block filter of each matrix (never on a diagonal block)."""
    X = C.copy() if square else (2.0 * (old if old is not None else 0.0) - C)
    if not diag and eps > 0.0:
        for m in range(X.shape[0]):
            if np.sqrt(np.sum(X[m] * X[m])) < eps:
                X[m] = 0.0
    return X


def old_block(X: Rows, I: int, J: int) -> Optional[np.ndarray]:
    cols, vals = X[I]
    p = np.searchsorted(cols, J)
    return vals[p] if p < len(cols) and cols[p] == J else None


def row_products(X: Rows, I: int) -> Tuple[np.ndarray, np.ndarray]:
    """Row I of X X and of X0 X1_d + X1_d X0, before the branch and the
    filter, by Gustavson's row-wise product (Algorithm 1): row I of the
    product is sum over K in row I of X_IK times row K.  Returns the columns J
    (sorted) and the blocks (len(J), 1 + D, b, b)."""
    cols, vals = X[I]
    rowsK = [X[int(K)] for K in cols]
    J = np.concatenate([r[0] for r in rowsK])              # every (K, J) pair of row I
    Bv = np.concatenate([r[1] for r in rowsK])             # X_K J blocks
    A = vals[np.repeat(np.arange(len(cols)), [len(r[0]) for r in rowsK])]   # X_I K blocks
    D = vals.shape[1] - 1
    PRODUCTS[0] += len(J) * (1 + 2 * D)
    P = np.empty_like(Bv)
    P[:, 0] = np.matmul(A[:, 0], Bv[:, 0])
    for d in range(D):
        P[:, 1 + d] = np.matmul(A[:, 0], Bv[:, 1 + d]) + np.matmul(A[:, 1 + d], Bv[:, 0])
    order = np.argsort(J, kind="stable")
    Jc, start = np.unique(J[order], return_index=True)
    return Jc, np.add.reduceat(P[order], start, axis=0)


def next_rows(X: Rows, square: bool, eps: float, rows: Iterable[int]) -> Rows:
    """Rows of the next iterate (one update of Eq. TC2 / TC2-CPSCF with the
    filter).  X must hold every row I asked for and every row K of it.

    Each block of row I is computed in row I and filtered by its own norm.
    In exact arithmetic a lower block (J < I) is the transpose of the upper
    block (J, I), which the dense oracle's filter uses to decide both; the two
    norms differ by rounding only, so the decisions differ only for a norm
    within rounding of eps."""
    out: Rows = {}
    for I in rows:
        I = int(I)
        cols, vals = X[I]
        Jc, C = row_products(X, I)
        # the old blocks X_IJ where row I holds them (DOUBLE: 2 X - C)
        p = np.minimum(np.searchsorted(cols, Jc), len(cols) - 1)
        has = cols[p] == Jc
        old = np.zeros_like(C)
        old[has] = vals[p[has]]
        Y = C if square else 2.0 * old - C
        # filter of each matrix, never on the diagonal block
        if eps > 0.0:
            norms = np.sqrt(np.sum(Y * Y, axis=(2, 3)))            # (nJ, 1 + D)
            drop = (norms < eps) & (Jc != I)[:, None]
            Y[drop] = 0.0
        keep = (Jc == I) | np.any(Y != 0.0, axis=(1, 2, 3))
        out[I] = (Jc[keep].astype(np.int64), Y[keep])
    return out


def diag_blocks_next(X: Rows, square: bool, rows: Iterable[int]) -> Dict[int, np.ndarray]:
    """Diagonal blocks of the next iterate (never filtered): what Tr X0 and
    Tr X1_d of the next iterate need."""
    out = {}
    for I in rows:
        I = int(I)
        C = upper_block(X, I, I)
        out[I] = combine_and_filter(C, old_block(X, I, I), square, 0.0, True)
    return out


def trace0(diag: Dict[int, np.ndarray]) -> float:
    return float(sum(np.trace(v[0]) for v in diag.values()))


def coupling_graph(H) -> List[np.ndarray]:
    """Block columns of every row of H (the graph the patterns grow on)."""
    return [np.asarray(H.col[int(H.row_ptr[I]):int(H.row_ptr[I + 1])]) for I in range(H.nb)]


def ball(graph: List[np.ndarray], seeds: Iterable[int], radius: int) -> np.ndarray:
    """Rows within ``radius`` steps of the seeds in the coupling graph."""
    seen = set(int(s) for s in seeds)
    front = list(seen)
    for _ in range(radius):
        nxt = []
        for I in front:
            for J in graph[I]:
                J = int(J)
                if J not in seen:
                    seen.add(J)
                    nxt.append(J)
        front = nxt
    return np.array(sorted(seen), dtype=np.int64)


@dataclass
class Leading:
    """Result of the first updates of a solve (see leading_updates)."""
    emin: float
    emax: float
    branches: str                  # 'S' / 'D' of updates 1 .. n
    traces: List[float]            # Tr X0 of iterates 0 .. n-1 (each decides the next branch)
    rows: List[Rows]               # rows[k - 1]: the requested rows of X_k, k = 1 .. n
    full1: Rows                    # every row of X_1
    scalars1: dict                 # Tr X0, E0, Tr X1_d, Tr(X1_d H), Tr(X1_d H1_d) of X_1


def _scalars(X: Rows, H, H1s) -> dict:
    """Traces and band energies of a complete iterate (Sec. 2.2): Tr X0,
    E0 = Tr(X0 H), Tr X1_d, E1_d = Tr(X1_d H), alpha_d = Tr(X1_d H1_d)."""
    b, D = H.b, len(H1s)
    def tr_prod(Xm_rows, M, m):
        # Tr(X M) = sum over blocks (I, J) of <X_IJ, M_IJ> with M symmetric
        t = 0.0
        for I in range(M.nb):
            cols, vals = Xm_rows[I]
            for p in range(int(M.row_ptr[I]), int(M.row_ptr[I + 1])):
                J = int(M.col[p])
                q = np.searchsorted(cols, J)
                if q < len(cols) and cols[q] == J:
                    t += float(np.sum(vals[q][m] * np.asarray(M.val[p]).reshape(b, b)))
        return t
    tr = [0.0] * (1 + D)
    for I, (cols, vals) in X.items():
        q = np.searchsorted(cols, I)
        for m in range(1 + D):
            tr[m] += float(np.trace(vals[q][m]))
    return dict(tr_x0=tr[0], tr_x1=tr[1:], e0=tr_prod(X, H, 0),
                e1=[tr_prod(X, H, 1 + d) for d in range(D)],
                alpha=[tr_prod(X, H1s[d], 1 + d) for d in range(D)])


def leading_updates(H, H1s: Sequence, n_occ: int, eps: float, sample_rows: Sequence[int],
                    n_updates: int = 3) -> Leading:
    """The first n_updates (1..3) updates of a solve, with the branch of each
    update decided by the trace rule (Tr X0 >= N_occ -> SQUARE) on the
    oracle's own iterates, and complete block rows ``sample_rows`` of every
    iterate X_1 .. X_n.  X_1 is computed in full; X_2 on the rows its sampled
    rows and X_3 need; X_3 on the sampled rows only."""
    assert 1 <= n_updates <= 3
    emin, emax = gershgorin_rows(H)
    graph = coupling_graph(H)
    all_rows = range(H.nb)
    X0 = init_rows(H, H1s, emin, emax)
    traces = [trace0({I: X0[I][1][np.searchsorted(X0[I][0], I)] for I in all_rows})]
    branches = "S" if traces[0] >= n_occ else "D"
    X1 = next_rows(X0, branches[0] == "S", eps, all_rows)
    out_rows = [{int(I): X1[int(I)] for I in sample_rows}]
    sc1 = _scalars(X1, H, H1s)
    if n_updates >= 2:
        traces.append(sc1["tr_x0"])
        branches += "S" if traces[1] >= n_occ else "D"
        sq2 = branches[1] == "S"
        # rows of X_2 needed: the sampled rows and, for a third update, the
        # rows K of the sampled rows of X_2 (X_2 couples rows up to 4 steps
        # apart in the coupling graph)
        need2 = ball(graph, sample_rows, 4) if n_updates >= 3 else np.asarray(sample_rows)
        X2 = next_rows(X1, sq2, eps, need2)
        out_rows.append({int(I): X2[int(I)] for I in sample_rows})
        if n_updates >= 3:
            tr2 = trace0(diag_blocks_next(X1, sq2, all_rows))
            traces.append(tr2)
            branches += "S" if tr2 >= n_occ else "D"
            X3 = next_rows(X2, branches[2] == "S", eps, sample_rows)
            out_rows.append(X3)
    return Leading(emin, emax, branches, traces, out_rows, X1, sc1)
