"""Write the oracle's results for the full-size workloads used by the GPU
parity tests (scalars and a seeded sample of blocks).  Calls only oracle/ and
the seeded input generator; run it on the CPU:

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
               blocks=[dict(I=i, J=j, X0=blk(r.X0, i, j), X1=[blk(x, i, j) for x in r.X1])
                       for i, j in pairs])
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: {r.iters} updates {r.branches} alpha={r.alpha} in {dt:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cube10")
