"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Both sides run the same recursion in FP64 with different summation orders,
so iterates agree to rounding (~1e-13) unless a block norm lies within
rounding of eps; the bar is the stated one, max|dX1| < 1e-6 and
rel|d alpha| < 1e-6, and the FP64 cases are held to 1e-9 / 1e-10 here.
"""
import numpy as np
import pytest

from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_X = 1e-9
FP64_A = 1e-10


def compare(sys, g, o, tol_x=FP64_X, tol_a=FP64_A, branches=True):
    print(f"  {sys.name}: gpu {g.status_name} it={g.iters} {g.branches} | "
          f"oracle st={o.status} it={o.iters} {o.branches}", flush=True)
    if branches:
        assert g.branches == o.branches
    dx0 = np.abs(T.bsr_dense(g.X0) - o.X0).max()
    assert dx0 < tol_x, dx0
    for d in range(len(sys.H1)):
        dx1 = np.abs(T.bsr_dense(g.X1[d]) - o.X1[d]).max()
        dal = abs(g.alpha[d] - o.alpha[d]) / max(abs(o.alpha[d]), 1e-300)
        print(f"    dir {d}: max|dX1|={dx1:.2e} rel|dalpha|={dal:.2e} alpha={g.alpha[d]:.10f}",
              flush=True)
        assert dx1 < tol_x, dx1
        assert dal < tol_a, dal
    assert abs(g.tr_x0 - np.trace(o.X0)) < 1e-8


def run_both(sys, **kw):
    g = T.solve(sys, **kw)[0]
    o = O.solve_system(sys)
    return g, o


KERNELS = ["tile", "block"]


@pytest.mark.parametrize("kernel", KERNELS)
def test_chain64_fp64(kernel):
    s = W.config_system("chain64")
    g, o = run_both(s, kernel=kernel)
    assert g.status == o.status == 0
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_chain_ragged_block(kernel):
    # b = 5 (one K-step of the padded tile is ragged), 37 atoms (ragged last cluster)
    s = W.config_system("chain64", n=37, b=5, occ=2, eps=1e-6, seed=17)
    g, o = run_both(s, kernel=kernel)
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_cube_b13_fp64(kernel):
    s = W.config_system("cube10", L=4)
    g, o = run_both(s, kernel=kernel)
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_purification_without_directions(kernel):
    # D = 0: X0 alone (TC2 without the response)
    s = W.config_system("cube10", L=4, n_dir=0)
    g, o = run_both(s, kernel=kernel)
    assert g.X1 == [] and g.alpha == []
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("b,occ", [(16, 6), (2, 1)])
def test_block_size_extremes(kernel, b, occ):
    # b = 16 fills the MFMA tile with no padding (four full K-steps); b = 2
    # uses one ragged K-step of a mostly empty tile
    s = W.config_system("chain64", n=29, b=b, occ=occ, eps=1e-6, seed=23)
    g, o = run_both(s, kernel=kernel)
    compare(s, g, o)


@pytest.mark.parametrize("b,occ", [(16, 6), (2, 1)])
def test_block_size_extremes_fp32_wide(b, occ):
    from oracle import exact as E
    s = W.config_system("chain64", n=29, b=b, occ=occ, eps=1e-9, seed=23)
    g = T.solve(s, precision="fp32", wide=True, closing_fp64=2, fp64_first=2)[0]
    H = O.bsr_to_dense(s.H.nb, s.H.b, s.H.row_ptr, s.H.col, s.H.val)
    H1 = O.bsr_to_dense(s.H1[0].nb, b, s.H1[0].row_ptr, s.H1[0].col, s.H1[0].val)
    dx1 = np.abs(T.bsr_dense(g.X1[0]) - E.exact_response(H, H1, s.n_occ)).max()
    dal = abs(g.alpha[0] - E.exact_alpha(H, H1, s.n_occ)) / abs(E.exact_alpha(H, H1, s.n_occ))
    print(f"  b={b}: {g.status_name} it={g.iters} max|dX1| {dx1:.2e} rel|dalpha| {dal:.2e}",
          flush=True)
    assert g.status >= 0 and dx1 < 1e-6 and dal < 1e-6


def test_cube_clusters_without_positions():
    # clusters taken in index order when no positions are given
    s = W.config_system("cube10", L=4)
    g, o = run_both(s, use_xyz=False)
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_cube_three_directions(kernel):
    s = W.config_system("cube20", L=3, eps=1e-6)
    g, o = run_both(s, kernel=kernel)
    compare(s, g, o)


def test_cube_two_directions_odd_lattice():
    s = W.config_system("cube20", L=5, n_dir=2, eps=1e-5)
    g, o = run_both(s)
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_batch_uneven_systems(kernel):
    sys_list = W.batch_systems(sizes=[20, 64, 9, 41], n_dir=2)
    gs = T.solve(sys_list, kernel=kernel)
    for s, g in zip(sys_list, gs):
        compare(s, g, O.solve_system(s))


def test_replay_branches():
    s = W.config_system("chain64", n=20)
    o = O.solve_system(s)
    rep = o.branches[:-3] + ("S" if o.branches[-3] == "D" else "D") + o.branches[-2:]
    g = T.solve(s, replay=[rep])[0]
    o2 = O.solve_system(s, replay=rep)
    assert g.branches == rep
    compare(s, g, o2)


@pytest.mark.parametrize("which", ["none", "all"])
def test_nocc_edges(which):
    s = W.config_system("chain64", n=5)
    s.n_occ = 0 if which == "none" else s.H.n
    g = T.solve(s)[0]
    X0 = T.bsr_dense(g.X0)
    assert g.status == 0 and g.iters == 0
    assert np.array_equal(X0, np.zeros_like(X0) if which == "none" else np.eye(X0.shape[0]))
    assert not np.any(T.bsr_dense(g.X1[0]))


def test_single_atom():
    s = W.config_system("chain64", n=1)
    g, o = run_both(s)
    compare(s, g, o)


def test_degenerate_spectrum():
    s = W.config_system("chain64", n=4, cutoff=0.5)
    s.H.val = np.broadcast_to(np.eye(8) * 0.3, s.H.val.shape).copy()
    with pytest.raises(T.TC2Error) as e:
        T.solve(s)
    assert e.value.status == -5


def test_max_iter_not_converged():
    s = W.config_system("chain64", n=16)
    s.max_iter = 3
    g = T.solve(s)[0]
    assert g.status == 1 and g.iters == 3
    o = O.solve_system(s, max_iter=3)
    compare(s, g, o)


def test_repeat_run_is_bitwise_identical():
    s = W.config_system("cube10", L=3)
    solver = T.Solver(s)
    a = solver.run()[0]
    b = solver.run()[0]
    solver.close()
    assert a.branches == b.branches
    assert np.array_equal(a.X1[0].val, b.X1[0].val)
    assert np.array_equal(a.X0.col, b.X0.col)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_norm_bound_screen_is_exact(prec):
    # the screen only skips blocks that the drop would remove: identical results
    s = W.config_system("cube10", L=5, eps=1e-5)
    a = T.solve(s, precision=prec)[0]
    b = T.solve(s, precision=prec, skip="bound")[0]
    print(f"  screened {b.screened_blocks} output blocks over {b.iters} updates", flush=True)
    assert b.screened_blocks > 0
    assert a.branches == b.branches
    assert np.array_equal(a.X0.col, b.X0.col)
    assert np.array_equal(a.X0.val, b.X0.val)
    assert np.array_equal(a.X1[0].val, b.X1[0].val)
    assert a.alpha == b.alpha


def test_norm_bound_screen_three_directions_matches_oracle():
    s = W.config_system("cube20", L=3, eps=1e-5)
    g, o = run_both(s, skip="bound")
    compare(s, g, o)


@pytest.fixture
def knob(monkeypatch):
    def set_(name, value):
        monkeypatch.setenv(name, str(value))
    return set_


@pytest.mark.parametrize("dirs,skip", [(1, "none"), (3, "none"), (3, "bound")])
def test_forced_multipass_panels(knob, dirs, skip):
    # panel passes of 64 columns: the path taken by large systems
    knob("TC2_TEST_KL_CHUNK", 64)
    s = W.config_system("cube20", L=4, n_dir=dirs, eps=1e-6)
    g, o = run_both(s, skip=skip)
    compare(s, g, o)


@pytest.mark.parametrize("dirs", [1, 3])
def test_forced_stage_overflow(knob, dirs):
    # a stage of 16 blocks overflows at every update and is grown and retried
    knob("TC2_TEST_STAGE_CAP", 16)
    s = W.config_system("cube20", L=4, n_dir=dirs, eps=1e-6)
    g, o = run_both(s)
    compare(s, g, o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_nominal_flops_count_full_product_triples(kernel):
    # nominal flops: 2 b^3 (1 + 2D) per block triple (I, K, J) of the full
    # products on each update's input pattern, i.e. the sum over rows K of
    # m_K^2 for the union block pattern of X0 and X1 (an integer count, exact)
    s = W.config_system("cube10", L=4)
    g = T.solve(s, kernel=kernel, count_useful=True)[0]
    b, D = s.H.b, len(s.H1)
    H = O.bsr_to_dense(s.H.nb, b, s.H.row_ptr, s.H.col, s.H.val)
    H1 = [O.bsr_to_dense(m.nb, b, m.row_ptr, m.col, m.val) for m in s.H1]
    emin, emax = O.gershgorin(H)
    X0, X1 = O.tc2_init(H, H1, emin, emax)
    nb = s.H.nb
    total = 0
    for br in g.branches:
        blocks = [X.reshape(nb, b, nb, b) for X in [X0] + X1]
        pat = np.zeros((nb, nb), dtype=bool)
        for B in blocks:
            pat |= np.abs(B).sum(axis=(1, 3)) > 0
        total += int((pat.sum(axis=1) ** 2).sum())
        X0, X1 = O.tc2_step(X0, X1, br == "S")
        X0 = O.block_drop(X0, b, s.eps)
        X1 = [O.block_drop(x, b, s.eps) for x in X1]
    want = total * 2.0 * b ** 3 * (1 + 2 * D)
    print(f"  nominal {g.nominal_flops:.6e} oracle {want:.6e} useful {g.useful_flops:.6e}", flush=True)
    assert g.nominal_flops == want
    assert g.nominal_flops > g.union_flops >= g.useful_flops > 0


@pytest.mark.parametrize("variant", [dict(precision="fp64"), dict(precision="fp64", kernel="block"),
                                     dict(precision="fp32", wide=True, fp64_first=2, closing_fp64=2,
                                          skip="bound", graph=True),
                                     dict(precision="bf16", closing_fp64=2)])
def test_zero_block_products_are_not_issued(knob, variant):
    # products with a block that is zero for its matrix (the union pattern
    # stores such blocks) add exact zeros: leaving them out changes no bit of
    # the result, and issues fewer products
    s = W.config_system("cube10", L=4, n_dir=3, eps=1e-5)
    a = T.solve(s, **variant)[0]
    knob("TC2_TEST_NO_ZERO_SKIP", 1)
    b = T.solve(s, **variant)[0]
    print(f"  executed {a.executed_flops / 1e9:.2f} GF with the masks, {b.executed_flops / 1e9:.2f} "
          f"without", flush=True)
    assert a.branches == b.branches and a.alpha == b.alpha
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.col, y.col) and np.array_equal(x.val, y.val)
    if variant.get("kernel") != "block":
        assert a.executed_flops < b.executed_flops


@pytest.mark.parametrize("case", [
    dict(name="cube10", kw=dict(L=5, n_dir=3, eps=1e-5), variant=dict(precision="fp64")),
    dict(name="cube10", kw=dict(L=5, n_dir=2, eps=1e-5),
         variant=dict(precision="fp64", skip="bound", graph=True)),
    dict(name="cube20", kw=dict(L=4, n_dir=3, eps=1e-6), variant=dict(precision="fp64"), chunk=64),
    dict(name="cube10", kw=dict(L=5, n_dir=3, eps=1e-5),
         variant=dict(precision="fp32", wide=True, fp64_first=2, closing_fp64=2, skip="bound",
                      graph=True)),
    dict(name="cube10", kw=dict(L=5, n_dir=3, eps=1e-5),
         variant=dict(precision="bf16", wide=True, fp64_first=2, closing_fp64=2, skip="bound")),
    # more cluster pairs than compute units: the FP64 kind keeps its 8x8 sub-tile
    dict(name="cube10", kw=dict(L=7, eps=1e-5),
         variant=dict(precision="fp64", skip="bound", graph=True)),
    dict(name="cube10", kw=dict(L=5),
         variant=dict(precision="fp32", wide=True, fp64_first=2, closing_fp64=2, skip="bound")),
])
def test_more_waves_per_column_equal_one(knob, case):
    # the 4x4 sub-tile with two or three directions runs four waves per
    # sub-tile column, the 8x8 sub-tile with one direction two (FP64 and the
    # kinds with FP64 sums); every output sums the same products in the same order
    # as with one wave per column, so the iterates are bitwise identical (only
    # the grouping of the per-workgroup trace sums differs)
    if "chunk" in case:
        knob("TC2_TEST_KL_CHUNK", case["chunk"])
    s = W.config_system(case["name"], **case["kw"])
    a = T.solve(s, **case["variant"])[0]
    knob("TC2_TEST_WAVES_PER_COLUMN", 1)
    b = T.solve(s, **case["variant"])[0]
    print(f"  {case['name']}: {a.iters} updates {a.branches}", flush=True)
    assert a.branches == b.branches and a.iters == b.iters
    for x, y in zip([a.X0] + a.X1, [b.X0] + b.X1):
        assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
        assert np.array_equal(x.val, y.val)
    for p, q in zip(a.alpha, b.alpha):
        assert p == pytest.approx(q, rel=1e-12)
