"""The exact count of useful block products (count_useful) against the
oracle's definition, update by update, on the oracle's own iterates.

The GPU counts on the device: per-entry masks of the nonzero matrices before
and after an update, and for every kept output the common columns of the
old rows.  The oracle counts with products of block-presence matrices of its
dense iterates (pinned against a triple loop).  Both sides follow the same
branches (the oracle replays the GPU's branch string); the counts are
integers and must be equal."""
import numpy as np
import pytest

from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def dense(m):
    return O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val)


def oracle_counts(s, branches):
    """Useful products of every update of the oracle's solve along
    ``branches``."""
    H, H1s = dense(s.H), [dense(h) for h in s.H1]
    b = s.H.b
    X0, X1s = O.tc2_init(H, H1s, *O.gershgorin(H))
    out = []
    for c in branches:
        N0, N1s = O.tc2_step(X0, X1s, c == "S")
        N0 = O.block_drop(N0, b, s.eps)
        N1s = [O.block_drop(x, b, s.eps) for x in N1s]
        out.append(O.useful_products([X0] + X1s, [N0] + N1s, b))
        X0, X1s = N0, N1s
    return out


@pytest.mark.parametrize("name,kw,variant", [
    ("chain64", dict(n=24), dict(precision="fp64")),
    ("chain64", dict(n=24), dict(precision="fp64", kernel="block")),
    ("cube10", dict(L=4, n_dir=3), dict(precision="fp64", graph=True, skip="bound")),
    ("cube10", dict(L=4, n_dir=1, eps=1e-5), dict(precision="fp64", graph=True)),
])
def test_count_per_update_equals_the_oracle(name, kw, variant):
    s = W.config_system(name, **kw)
    b3 = 2.0 * s.H.b ** 3
    sv = T.Solver(s, count_useful=True, **variant)
    try:
        per = []
        while True:
            p, r = sv.advance(1)
            if p["updates"]:
                per.append(p["useful_flops"] / b3)
            if r is not None:
                g = r[0]
                break
    finally:
        sv.close()
    want = oracle_counts(s, g.branches)
    print(f"  {name}: {g.branches} per-update products {per[:6]}...", flush=True)
    assert per == want
    assert g.useful_flops == b3 * sum(want)
    assert g.useful_flops_kind[0] == g.useful_flops
    # the union-pattern count is an upper bound of it
    assert g.union_flops >= g.useful_flops > 0


def test_count_per_system_of_a_batch():
    systems = W.batch_systems(n_sys=3, lo=30, hi=80, seed=5, n_dir=2)
    g = T.solve(systems, precision="fp64", count_useful=True)
    for sy, r in zip(systems, g):
        want = oracle_counts(sy, r.branches)
        assert r.useful_flops == 2.0 * sy.H.b ** 3 * sum(want)


def test_count_of_the_benchmarked_variant_by_kind():
    # FP64 first, then FP32 with FP64 sums, then the closing FP64 pair: the
    # counts land under the kind of each update and add up to the total
    s = W.config_system("cube10", L=4, n_dir=3)
    g = T.solve(s, precision="fp32", wide=True, fp64_first=4, closing_fp64=2, skip="bound",
                graph=True, count_useful=True)[0]
    k = g.useful_flops_kind
    assert k[0] > 0 and k[3] > 0 and k[1] == k[2] == 0
    assert k[0] + k[3] == g.useful_flops
