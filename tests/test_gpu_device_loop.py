"""Branch and stopping decisions taken on the device (device_loop = k) against
the same solves with the decisions on the host (graph = 1): identical status,
branch string and update count, bit-identical X0 / X1 and counters, and the
device path is the one that ran.  Both run the same update graphs; the device
loop adds the decision kernel at the end of each and copies the iterate of a
stopped system through on the updates it replays after the last stop."""
import numpy as np
import pytest

from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def same(a, b):
    assert a.status == b.status and a.branches == b.branches and a.iters == b.iters
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)
    assert a.alpha == b.alpha and a.e0 == b.e0 and a.tr_x0 == b.tr_x0
    assert a.union_flops == b.union_flops and a.nominal_flops == b.nominal_flops
    assert a.executed_flops == b.executed_flops and a.kept_blocks == b.kept_blocks
    assert a.screened_blocks == b.screened_blocks


def both(systems, k, **kw):
    ref = T.solve(systems, graph=True, **kw)
    got = T.solve(systems, graph=True, device_loop=k, **kw)
    for r, g in zip(ref, got):
        print(f"  k={k} {r.status_name} it={r.iters} {r.branches} device updates "
              f"{g.device_loop_updates}", flush=True)
        same(g, r)
    return ref, got


@pytest.mark.parametrize("k", [1, 3, 64])
def test_device_decisions_chain(k):
    s = W.config_system("chain64")
    _, got = both(s, k)
    assert got[0].device_loop_updates == got[0].iters > 0


@pytest.mark.parametrize("variant", [dict(), dict(skip="bound")])
def test_device_decisions_cube_three_directions(variant):
    s = W.config_system("cube10", L=5)
    _, got = both(s, 4, **variant)
    assert got[0].device_loop_updates == got[0].iters


def test_device_decisions_batch_with_systems_stopping_apart():
    # uneven systems stop at different updates; the device clears their
    # flags and the later updates copy them through
    systems = W.batch_systems(n_sys=4, sizes=[30, 64, 100, 45], n_dir=1)
    ref, got = both(systems, 5, skip="bound")
    assert len({r.iters for r in ref}) > 1
    assert all(g.device_loop_updates == max(r.iters for r in ref) for g in got)


@pytest.mark.parametrize("case", ["single_atom", "max_iter", "ragged_chain", "mixed_batch",
                                  "no_direction", "first_update_stop", "many_systems"])
def test_device_decisions_edge_cases(case):
    if case == "single_atom":
        systems = W.config_system("chain64", n=1)
    elif case == "no_direction":
        systems = W.config_system("chain64", n=20, n_dir=0)
    elif case == "first_update_stop":
        # max_iter = 1 stops one system after its first update, beside others
        a = W.config_system("chain64", n=12)
        a.max_iter = 1
        systems = [a, W.config_system("chain64", n=9), W.config_system("chain64", n=16, seed=9)]
    elif case == "many_systems":
        # more systems than the decision kernel's 256 threads (its stride loop)
        systems = [W.config_system("chain64", n=2 + k % 3, seed=100 + k) for k in range(300)]
    elif case == "max_iter":
        systems = W.config_system("chain64", n=16)
        systems.max_iter = 3
    elif case == "ragged_chain":
        systems = W.config_system("chain64", n=23, b=5)
    else:
        # a trivial system (N_occ = N) next to iterating ones of different sizes
        a = W.config_system("chain64", n=6)
        a.n_occ = a.H.n
        systems = [a, W.config_system("chain64", n=17), W.config_system("chain64", n=30)]
    ref, got = both(systems, 2)
    if case == "max_iter":
        assert ref[0].status_name == "NOT_CONVERGED" and ref[0].iters == 3
    if case == "first_update_stop":
        assert ref[0].iters == 1 and ref[1].iters > 1
    if case != "single_atom":
        assert max(g.device_loop_updates for g in got) == max(r.iters for r in ref) > 0


def test_device_decisions_repeated_runs_replay_their_graphs():
    s = W.config_system("cube10", L=4)
    solver = T.Solver(s, graph=True, device_loop=4)
    a = solver.run()[0]
    b = solver.run()[0]
    solver.close()
    same(a, b)
    print(f"  captures {a.graph_captures} then {b.graph_captures}", flush=True)
    assert a.device_loop_updates == a.iters and b.device_loop_updates == b.iters
    assert a.graph_captures <= 2 and b.graph_captures == 0


@pytest.mark.parametrize("variant", [dict(replay=["SDSDDSDSDS"]),
                                     dict(precision="fp32", closing_fp64=2, wide=True),
                                     dict(count_useful=True)])
def test_device_decisions_fall_back_to_the_host(variant):
    # outside the device loop's scope the host decides, with the same results
    s = W.config_system("chain64", n=20)
    ref = T.solve(s, graph=True, **variant)[0]
    got = T.solve(s, graph=True, device_loop=4, **variant)[0]
    same(got, ref)
    assert got.device_loop_updates == 0


@pytest.mark.parametrize("case", ["chain", "cube_three_directions"])
def test_device_decisions_against_the_oracle(case):
    # the device's branches, update count and status against the oracle's
    # own rule, and X1 and alpha against the oracle's iterate
    from oracle import tc2_oracle as O
    s = (W.config_system("chain64", n=24) if case == "chain"
         else W.config_system("cube10", L=3, n_dir=3))
    g = T.solve(s, graph=True, skip="bound", device_loop=3)[0]
    o = O.solve_system(s)
    print(f"  {case}: {g.status_name} it={g.iters} {g.branches} (oracle {o.branches})", flush=True)
    assert g.device_loop_updates == g.iters
    assert g.branches == o.branches and g.iters == len(o.branches) and g.status == o.status
    for d in range(len(s.H1)):
        assert np.abs(T.bsr_dense(g.X1[d]) - o.X1[d]).max() < 1e-9
        assert abs(g.alpha[d] - o.alpha[d]) <= 1e-10 * abs(o.alpha[d])
