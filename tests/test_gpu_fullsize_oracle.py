"""Full-size parity against the block-list oracle: the first three updates of
cube20 (8000 atoms, N = 104000, three directions), cube30 (27000 atoms,
N = 351000, three directions, eps 1e-5) and one unit of the batch of 32
systems, on complete sampled block rows of every iterate.

The GPU runs one update at a time (tc2_advance) with its own branch
decisions, and exports the sampled rows after each (tc2_export_rows).  The
oracle (oracle/bsr_oracle.py, plain FP64 block lists) computes the same
rows, deciding its branches from its own traces.  Both sides are FP64 in
these updates, in both the plain path and the benchmarked variant (whose
first four updates are FP64, with the exact screen and update graphs), so
the rows agree to rounding; the bar is 1e-9 per element and identical block
patterns.
"""
import numpy as np
import pytest

from oracle import bsr_oracle as B
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = {
    "plain_fp64": dict(precision="fp64", graph=True),
    "bench": dict(precision="fp32", wide=True, fp64_first=4, closing_fp64=2, skip="bound",
                  graph=True),
}
TOL = 1e-9
_cache = {}


def workload(name):
    """Systems of the workload, their sampled rows and the oracle's rows."""
    if name in _cache:
        return _cache[name]
    if name == "batch32_unit":
        systems = W.pack_units(W.batch_systems(), 16000)[0]
    else:
        systems = [W.config_system(name)]
    rows, leads = [], []
    for s in systems:
        nb = s.H.nb
        r = sorted({0, nb // 2 + 7 if nb > 20 else nb // 2, nb - 1})
        rows.append(r)
        leads.append(B.leading_updates(s.H, s.H1, s.n_occ, s.eps, r, n_updates=3))
    print(f"  oracle for {name}: {len(systems)} system(s), branches "
          f"{[l.branches for l in leads]}", flush=True)
    _cache[name] = (systems, rows, leads)
    return _cache[name]


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("name", ["cube20", "cube30", "batch32_unit"])
def test_leading_updates_match_the_block_oracle(name, variant):
    systems, rows, leads = workload(name)
    print(f"  {name} / {variant}: atoms {sum(s.H.nb for s in systems)}", flush=True)
    sv = T.Solver(systems, export=False, **VARIANTS[variant])
    try:
        for k in (1, 2, 3):
            p, r = sv.advance(1)
            assert p["updates"] == 1 and r is None
            worst = 0.0
            for sidx, (s, rr, lead) in enumerate(zip(systems, rows, leads)):
                x0, x1 = sv.export_rows(sidx, rr)
                mats = [x0] + x1
                for I in rr:
                    ocols, ovals = lead.rows[k - 1][I]
                    a0, a1 = int(x0.row_ptr[I]), int(x0.row_ptr[I + 1])
                    assert np.array_equal(x0.col[a0:a1], ocols), (name, k, I)
                    for m, X in enumerate(mats):
                        d = np.abs(X.val[a0:a1] - ovals[:, m]).max()
                        worst = max(worst, d)
            print(f"    update {k}: max |gpu - oracle| over sampled rows {worst:.2e}", flush=True)
            assert worst < TOL
    finally:
        sv.close()
