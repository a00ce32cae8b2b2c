"""Write the oracle's results for the full-size workloads used by the GPU
parity tests: the scalars of every update (Tr X0, E0, E1_d, alpha_d, iota),
a seeded sample of blocks, and complete block rows of the final X0 and X1_d
(a corner, an edge and the centre atom of the cube) in <name>_rows.npz.
Calls only oracle/ and the seeded input generator; run it on the CPU:

    python tests/golden/make_golden.py cube10      # about 15 min on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tc2_oracle as O  # noqa: E402
from paper_2009_03551_amd import workloads as W  # noqa: E402


def sample_pairs(nb, X0, b, rng, n_near=24, n_far=8):
    """Upper blocks to store: some kept near the diagonal, some far."""
    blocks = X0.reshape(nb, b, nb, b)
    nrm = np.sqrt(np.einsum("iajb,iajb->ij", blocks, blocks))
    I, J = np.nonzero(np.triu(nrm > 0))
    pick = rng.choice(len(I), size=min(n_near, len(I)), replace=False)
    pairs = [(int(I[k]), int(J[k])) for k in pick]
    for _ in range(n_far):
        i, j = sorted(rng.integers(0, nb, 2).tolist())
        pairs.append((i, j))
    return pairs


def full_rows(name, nb):
    """Atoms whose complete block rows are stored: a corner, an edge atom and
    the centre of the cube (or the two ends and the middle of a chain)."""
    L = round(nb ** (1.0 / 3.0))
    if L ** 3 == nb:
        h = L // 2
        return [0, h * L, h * L * L + h * L + h]          # (0,0,0), (0,h,0), (h,h,h)
    return [0, nb // 2, nb - 1]


def main(name):
    s = W.config_system(name)
    t0 = time.time()
    r = O.solve_system(s, keep_history=True)
    dt = time.time() - t0
    b, nb = s.H.b, s.H.nb
    rng = np.random.default_rng(12345)
    pairs = sample_pairs(nb, r.X0, b, rng)
    blk = lambda X, i, j: X[i * b:(i + 1) * b, j * b:(j + 1) * b].tolist()
    out = dict(workload=name, N=s.H.n, atoms=nb, b=b, n_occ=s.n_occ, eps=s.eps, tol=s.tol,
               status=r.status, iters=r.iters, branches=r.branches, alpha=r.alpha,
               emin=r.emin, emax=r.emax, tr_x0=float(np.trace(r.X0)),
               e0=r.history[-1]["E0"], e1=r.history[-1]["E1"],
               idem=r.history[-1]["iota"], oracle_seconds=dt,
               history=r.history,
               blocks=[dict(I=i, J=j, X0=blk(r.X0, i, j), X1=[blk(x, i, j) for x in r.X1])
                       for i, j in pairs])
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    # complete rows: every block (I, J) nonzero in X0 or some X1_d
    rows = full_rows(name, nb)
    mats = [r.X0] + list(r.X1)
    arrays = {}
    for I in rows:
        strip = np.stack([m[I * b:(I + 1) * b, :].reshape(b, nb, b).transpose(1, 0, 2) for m in mats],
                         axis=1)                                  # (nb, 1 + D, b, b)
        cols = np.nonzero(np.any(strip != 0.0, axis=(1, 2, 3)))[0]
        arrays[f"cols_{I}"] = cols.astype(np.int32)
        arrays[f"vals_{I}"] = strip[cols]
    arrays["rows"] = np.array(rows, dtype=np.int32)
    np.savez_compressed(os.path.join(HERE, f"{name}_rows.npz"), **arrays)
    print(f"wrote {path}: {r.iters} updates {r.branches} alpha={r.alpha} in {dt:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cube10")
