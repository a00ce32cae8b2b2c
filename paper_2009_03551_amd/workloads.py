"""Seeded synthetic inputs for the TC2 / TC2-CPSCF response solver.

This module only *draws* inputs: atom positions, a block-sparse Hamiltonian H
in an orthonormal basis, the electric-field perturbation H1 (position
operator), and the occupation count.  It holds none of the method's
arithmetic, so that both the CPU oracle and the GPU path can be fed the very
same matrices.

Recipe (stand-in for the paper's FHI-aims Hamiltonians of H(C2H4)nH chains
and molecules, Sec. 3, which are not available):

* atoms on a 1D chain or a simple-cubic lattice with spacing ``a``;
* ``b`` orbitals per atom; the onsite block is diagonal, -1 for the first
  ``occ_per_atom`` orbitals and +1 for the rest;
* for every unordered atom pair I < J with distance r <= cutoff, an off-site
  block with entries U(-amp, amp) * exp(-r / decay) is drawn (pairs in
  row-major (I, J) order, entries row-major), and H_JI = H_IJ^T;
* H1_d = blockdiag((x_{I,d} - mean_d) * 1_b), the position operator of the
  homogeneous field (Sec. 2) in the point-atom approximation, centred.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "BSR", "System", "chain_positions", "cubic_positions", "make_system",
    "config_system", "batch_systems", "CONFIGS",
]


@dataclass
class BSR:
    """Square block-sparse matrix with uniform b x b blocks.

    ``row_ptr`` (int64, nb+1), ``col`` (int32, nnzb, strictly increasing per
    row) and ``val`` (float64, nnzb x b x b, each block row-major).  The
    pattern is the full (both triangles) pattern.
    """
    nb: int
    b: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n(self) -> int:
        return self.nb * self.b


@dataclass
class System:
    H: BSR
    H1: List[BSR]
    n_occ: int
    xyz: np.ndarray            # (nb, 3) atom positions
    eps: float = 1e-6          # block drop threshold
    tol: float = 1e-9          # convergence tolerance
    max_iter: int = 100
    name: str = ""
    meta: dict = field(default_factory=dict)


def chain_positions(n_atoms: int, spacing: float = 1.0) -> np.ndarray:
    xyz = np.zeros((n_atoms, 3))
    xyz[:, 0] = spacing * np.arange(n_atoms)
    return xyz


def cubic_positions(L: int, spacing: float = 2.5, n_first: Optional[int] = None) -> np.ndarray:
    """Sites of an L x L x L simple-cubic lattice in row-major (x slowest)
    order; optionally only the first ``n_first`` of them."""
    g = np.arange(L, dtype=np.float64) * spacing
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if n_first is not None:
        xyz = xyz[:n_first]
    return np.ascontiguousarray(xyz)


def _pairs_within(xyz: np.ndarray, cutoff: float) -> np.ndarray:
    """All (I, J) with I < J and |x_I - x_J| <= cutoff, row-major order."""
    from scipy.spatial import cKDTree
    tree = cKDTree(xyz)
    # a tiny slack so that exact lattice distances equal to the cutoff count
    pairs = tree.query_pairs(cutoff * (1.0 + 1e-12), output_type="ndarray")
    if len(pairs) == 0:
        return np.zeros((0, 2), dtype=np.int64)
    pairs = np.sort(pairs, axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order].astype(np.int64)


def _assemble(nb: int, b: int, pairs: np.ndarray, offblocks: np.ndarray,
              diagblocks: np.ndarray) -> BSR:
    """Full symmetric-pattern BSR from diagonal blocks and upper off-site
    blocks (the lower ones are their transposes)."""
    npair = len(pairs)
    rows = np.concatenate([np.arange(nb), pairs[:, 0], pairs[:, 1]])
    cols = np.concatenate([np.arange(nb), pairs[:, 1], pairs[:, 0]])
    vals = np.concatenate([diagblocks, offblocks,
                           np.transpose(offblocks, (0, 2, 1))]) if npair else diagblocks
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return BSR(nb, b, row_ptr, cols.astype(np.int32),
               np.ascontiguousarray(vals, dtype=np.float64))


def make_system(xyz: np.ndarray, b: int, occ_per_atom: int, cutoff: float,
                seed: int, n_dir: int = 1, amp: float = 0.3,
                decay: float = 1.5, eps: float = 1e-6, tol: float = 1e-9,
                max_iter: int = 100, name: str = "") -> System:
    xyz = np.asarray(xyz, dtype=np.float64)
    nb = len(xyz)
    rng = np.random.default_rng(seed)
    pairs = _pairs_within(xyz, cutoff)
    r = np.linalg.norm(xyz[pairs[:, 0]] - xyz[pairs[:, 1]], axis=1) if len(pairs) else np.zeros(0)
    off = rng.uniform(-amp, amp, size=(len(pairs), b, b))
    off *= np.exp(-r / decay)[:, None, None]
    onsite = np.diag(np.concatenate([-np.ones(occ_per_atom), np.ones(b - occ_per_atom)]))
    diag = np.broadcast_to(onsite, (nb, b, b)).copy()
    H = _assemble(nb, b, pairs, off, diag)
    H1 = []
    centre = xyz.mean(axis=0)
    eye = np.eye(b)
    for d in range(n_dir):
        x = xyz[:, d] - centre[d]
        blocks = x[:, None, None] * eye[None, :, :]
        H1.append(BSR(nb, b, np.arange(nb + 1, dtype=np.int64),
                      np.arange(nb, dtype=np.int32), np.ascontiguousarray(blocks)))
    return System(H=H, H1=H1, n_occ=occ_per_atom * nb, xyz=xyz, eps=eps,
                  tol=tol, max_iter=max_iter, name=name,
                  meta=dict(b=b, occ_per_atom=occ_per_atom, cutoff=cutoff,
                            seed=seed, amp=amp, decay=decay))


def make_overlap(system: System, amp: float = 0.08, decay: float = 1.5, seed: int = 7,
                 min_disc: float = 0.2) -> BSR:
    """A synthetic overlap matrix S for a non-orthogonal basis: the pattern of
    H, unit diagonal blocks plus small symmetric on-site terms, and off-site
    blocks decaying with distance.  The off-site part is scaled down if
    needed so that every Gershgorin disc of S stays above ``min_disc``: S is
    symmetric positive definite."""
    H, xyz = system.H, system.xyz
    nb, b = H.nb, H.b
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(nb), np.diff(H.row_ptr))
    upper = [(int(i), int(j)) for i, j in zip(rows, H.col) if j > i]
    pairs = np.array(upper, dtype=np.int64).reshape(-1, 2)
    r = np.linalg.norm(xyz[pairs[:, 0]] - xyz[pairs[:, 1]], axis=1) if len(pairs) else np.zeros(0)
    off = rng.uniform(-amp, amp, size=(len(pairs), b, b)) * np.exp(-r / decay)[:, None, None]
    g = rng.uniform(-0.02, 0.02, size=(nb, b, b))
    diag = np.eye(b)[None] + 0.5 * (g + np.transpose(g, (0, 2, 1)))
    # Gershgorin discs of the scalar rows: centre S_ii, radius sum_j |S_ij|
    rad = np.abs(diag).sum(axis=2) - np.abs(np.diagonal(diag, axis1=1, axis2=2))
    rad_off = np.zeros((nb, b))
    if len(pairs):
        np.add.at(rad_off, pairs[:, 0], np.abs(off).sum(axis=2))
        np.add.at(rad_off, pairs[:, 1], np.abs(off).sum(axis=1))
    centre = np.diagonal(diag, axis1=1, axis2=2)
    worst = (centre - rad - rad_off).min()
    if worst < min_disc:
        slack = (centre - rad).min() - min_disc
        off *= max(slack, 0.0) / max(rad_off.max(), 1e-300)
    return _assemble(nb, b, pairs, off, diag)


def make_displacement(system: System, atom: int, amp_s: float = 0.05, amp_h: float = 0.2,
                      decay: float = 1.5, seed: int = 11):
    """Synthetic first-order matrices (H1, S1) of an atomic displacement: the
    basis functions of ``atom`` move, so both the Hamiltonian and the overlap
    change in the block row and column of that atom (blocks decaying with
    distance; the on-site overlap block does not change).  Returns two BSR
    matrices with the same symmetric pattern."""
    H, xyz = system.H, system.xyz
    nb, b = H.nb, H.b
    rng = np.random.default_rng(seed)
    nbrs = [int(j) for j in H.col[H.row_ptr[atom]:H.row_ptr[atom + 1]] if j != atom]
    pairs = np.array([(min(atom, j), max(atom, j)) for j in nbrs], dtype=np.int64).reshape(-1, 2)
    r = np.linalg.norm(xyz[pairs[:, 0]] - xyz[pairs[:, 1]], axis=1) if len(pairs) else np.zeros(0)
    w = np.exp(-r / decay)[:, None, None]
    s_off = rng.uniform(-amp_s, amp_s, size=(len(pairs), b, b)) * w
    h_off = rng.uniform(-amp_h, amp_h, size=(len(pairs), b, b)) * w
    g = rng.uniform(-amp_h, amp_h, size=(b, b))
    h_diag = np.zeros((nb, b, b))
    h_diag[atom] = 0.5 * (g + g.T)
    s_diag = np.zeros((nb, b, b))

    def only(bsr):  # keep the blocks in the row or column of the atom
        rows = np.repeat(np.arange(nb), np.diff(bsr.row_ptr))
        keep = (rows == atom) | (bsr.col == atom)
        rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=nb))])
        return BSR(nb, b, rp.astype(np.int64), bsr.col[keep], bsr.val[keep])

    return only(_assemble(nb, b, pairs, h_off, h_diag)), only(_assemble(nb, b, pairs, s_off, s_diag))


# Named workloads: one JSON file each under configs/, holding the recipe
# parameters and the readings of what the paper leaves open for that workload
# (lattice spacing, occupation for b = 13, tolerances, batch geometry).
_CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def _load_configs() -> dict:
    out = {}
    for f in sorted(os.listdir(_CONFIG_DIR)):
        if f.endswith(".json"):
            with open(os.path.join(_CONFIG_DIR, f)) as fh:
                out[f[:-5]] = json.load(fh)
    return out


CONFIGS = _load_configs()


def config_system(name: str, **override) -> System:
    """Build a named workload; keyword overrides (e.g. ``L=4``) shrink it."""
    c = dict(CONFIGS[name])
    c.update(override)
    if c["kind"] == "chain":
        xyz = chain_positions(c["n"], c["spacing"])
    elif c["kind"] == "cube":
        xyz = cubic_positions(c["L"], c["spacing"], c.get("n_first"))
    else:
        raise ValueError(f"{name} is a batch: use batch_systems()")
    return make_system(xyz, c["b"], c["occ"], c["cutoff"], c["seed"],
                       n_dir=c["n_dir"], eps=c["eps"], tol=c["tol"],
                       name=name)


def pack_units(systems: Sequence[System], max_atoms: int) -> List[List[System]]:
    """Consecutive systems packed into units of at most ``max_atoms`` atoms
    (a single larger system forms a unit of its own), so that the iterates
    of one unit fit in device memory."""
    units: List[List[System]] = []
    cur: List[System] = []
    acc = 0
    for sy in systems:
        if cur and acc + sy.H.nb > max_atoms:
            units.append(cur)
            cur, acc = [], 0
        cur.append(sy)
        acc += sy.H.nb
    if cur:
        units.append(cur)
    return units


def batch_systems(n_sys: Optional[int] = None, lo: Optional[int] = None,
                  hi: Optional[int] = None, seed: Optional[int] = None,
                  b: Optional[int] = None, n_dir: Optional[int] = None,
                  eps: Optional[float] = None, tol: Optional[float] = None,
                  spacing: Optional[float] = None,
                  sizes: Optional[Sequence[int]] = None) -> List[System]:
    """Independent systems of uneven size (defaults: configs/batch32.json):
    n_k atoms drawn uniformly in [lo, hi]; system k is the first n_k sites
    (row-major) of the smallest cube holding them, with its own seed
    1000*seed + k."""
    c = CONFIGS["batch32"]
    n_sys = c["n_sys"] if n_sys is None else n_sys
    lo = c["lo"] if lo is None else lo
    hi = c["hi"] if hi is None else hi
    seed = c["size_seed"] if seed is None else seed
    b = c["b"] if b is None else b
    n_dir = c["n_dir"] if n_dir is None else n_dir
    eps = c["eps"] if eps is None else eps
    tol = c["tol"] if tol is None else tol
    spacing = c["spacing"] if spacing is None else spacing
    if sizes is None:
        sizes = np.random.default_rng(seed).integers(lo, hi + 1, n_sys)
    out = []
    for k, n in enumerate(sizes):
        n = int(n)
        L = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
        while L ** 3 < n:
            L += 1
        xyz = cubic_positions(L, spacing, n_first=n)
        out.append(make_system(xyz, b, c["occ"], c["cutoff"], 1000 * seed + k, n_dir=n_dir,
                               eps=eps, tol=tol, name=f"batch{k}"))
    return out
