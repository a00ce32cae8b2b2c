"""Updates captured as hipGraphs (persistent numeric launch, sizes on the
device) against the same solves without graphs: identical branch strings and
bit-identical X0 / X1 (the same kernels run on the same data; only the
sub-tile order of the persistent launch and the buffer sizes differ), and the
graph path is the one that ran."""
import numpy as np
import pytest

from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def same(a, b):
    assert a.status == b.status and a.branches == b.branches and a.iters == b.iters
    # the exact screen skips the same outputs: a captured update takes the
    # block norms of its iterate from the previous update's gather, an
    # update without a graph computes them itself (bitwise the same norms)
    assert a.screened_blocks == b.screened_blocks
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)
    for x, y in zip(a.alpha, b.alpha):
        assert abs(x - y) <= 1e-12 * abs(y)


def both(systems, **kw):
    ref = T.solve(systems, **kw)
    got = T.solve(systems, graph=True, **kw)
    for r, g in zip(ref, got):
        print(f"  {r.status_name} it={r.iters} graph updates {g.graph_updates}", flush=True)
        same(g, r)
    return ref, got


@pytest.mark.parametrize("variant", [dict(), dict(skip="bound"), dict(profile=True)])
def test_graph_fp64(variant):
    s = W.config_system("cube10", L=5)
    _, got = both(s, **variant)
    assert got[0].graph_updates == got[0].iters


def test_graph_fp32_wide_three_directions():
    s = W.config_system("cube20", L=3)
    _, got = both(s, precision="fp32", closing_fp64=2, fp64_first=2, wide=True, skip="bound")
    # the closing FP64 pair runs as direct launches
    assert got[0].graph_updates == got[0].iters - 2


def test_graph_bf16_stages():
    s = W.config_system("cube20", L=3, n_dir=1)
    _, got = both(s, precision="bf16", closing_fp64=2)
    assert got[0].graph_updates == got[0].iters - 2


def test_graph_batch_with_stopped_systems():
    # uneven systems stop at different updates: the later updates copy the
    # stopped ones through inside the graph
    systems = W.batch_systems(n_sys=4, sizes=[30, 64, 100, 45], n_dir=1)
    _, got = both(systems, skip="bound")
    assert all(g.graph_updates > 0 for g in got)


def test_graph_stage_overflow(monkeypatch):
    # a 16-block stage overflows at every update: grown, re-captured, rerun
    monkeypatch.setenv("TC2_TEST_STAGE_CAP", "16")
    s = W.config_system("cube10", L=4)
    _, got = both(s)
    assert got[0].graph_updates == got[0].iters


def test_graph_repeated_runs_are_bitwise_identical():
    s = W.config_system("cube10", L=5)
    solver = T.Solver(s, graph=True, skip="bound")
    a = solver.run()[0]
    b = solver.run()[0]
    solver.close()
    same(a, b)
    assert a.graph_updates == a.iters and b.graph_updates == b.iters


@pytest.mark.parametrize("case", ["single_atom", "max_iter", "replay", "ragged_chain", "mixed_batch"])
def test_graph_edge_cases(case):
    # the graph path on the inputs the parity tests use for edge cases
    if case == "single_atom":
        systems, kw = W.config_system("chain64", n=1), {}
    elif case == "max_iter":
        s = W.config_system("chain64", n=16)
        s.max_iter = 3
        systems, kw = s, {}
    elif case == "replay":
        systems, kw = W.config_system("chain64", n=20), dict(replay=["SDSDDSDSDSDS"])
    elif case == "ragged_chain":
        systems, kw = W.config_system("chain64", n=23, b=5), {}
    else:
        # a trivial system (N_occ = N) next to iterating ones of different sizes
        a = W.config_system("chain64", n=6)
        a.n_occ = a.H.n
        systems, kw = [a, W.config_system("chain64", n=17), W.config_system("chain64", n=30)], {}
    ref, got = both(systems, **kw)
    assert any(g.graph_updates > 0 for g in got) or all(r.iters == 0 for r in ref)


def test_graph_is_replayed_once_the_pattern_settles():
    # the capacity in the graph key is rounded up to geometric buckets, so the
    # updates after the pattern stops growing replay a captured graph
    s = W.config_system("cube10", L=6, n_dir=1)
    g = T.solve(s, precision="fp32", wide=True, fp64_first=4, closing_fp64=2, skip="bound",
                graph=True)[0]
    print(f"  {g.iters} updates, {g.graph_updates} as graphs, {g.graph_captures} captures",
          flush=True)
    assert g.graph_updates >= g.iters - 2            # the closing pair runs without graphs
    assert 0 < g.graph_captures < g.graph_updates
