"""The dense O(N^3) path (tc2_dense_response: eigenpairs by rocSOLVER,
products by rocBLAS, HIP kernels for the rest) against the oracle's closed
forms (dense diagonalisation on the CPU), its edge cases, and its agreement
with the linear-scaling path."""
import numpy as np
import pytest

from oracle import exact as E
from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def dense_inputs(s):
    H = O.bsr_to_dense(s.H.nb, s.H.b, s.H.row_ptr, s.H.col, s.H.val)
    H1 = [O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val) for m in s.H1]
    return H, H1


CASES = {
    "chain64": lambda: W.config_system("chain64", n=24),
    "ragged_b5": lambda: W.config_system("chain64", n=23, b=5),
    "cube_b13": lambda: W.config_system("cube10", L=4),
    "three_dirs": lambda: W.config_system("cube20", L=3),
    "no_dirs": lambda: W.config_system("cube10", L=3, n_dir=0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_dense_matches_oracle(case):
    s = CASES[case]()
    H, H1 = dense_inputs(s)
    r = T.dense_response(s, export=True)
    print(f"  {case}: N={H.shape[0]} gap={r.gap:.3e} eigh {r.ms_eigh:.1f} ms "
          f"P1 {r.ms_p1:.1f} ms", flush=True)
    assert r.status == 0
    e = np.linalg.eigvalsh(H)
    np.testing.assert_allclose(r.eigenvalues, e, atol=1e-12 * np.abs(e).max())
    assert abs(r.gap - (e[s.n_occ] - e[s.n_occ - 1])) < 1e-12 * np.abs(e).max()
    P0 = E.exact_projector(H, s.n_occ)
    assert np.abs(r.P0 - P0).max() < 1e-11
    assert np.array_equal(r.P0, r.P0.T)                  # mirrored, exactly symmetric
    assert abs(r.tr_p0 - s.n_occ) < 1e-9 * s.n_occ
    assert abs(r.e0 - np.sum(P0 * H)) < 1e-11 * abs(r.e0)
    for d in range(len(s.H1)):
        P1 = E.exact_response(H, H1[d], s.n_occ)
        scale = np.abs(P1).max()
        assert np.abs(r.P1[d] - P1).max() < 1e-10 * scale, d
        a = E.exact_alpha(H, H1[d], s.n_occ)
        assert abs(r.alpha[d] - a) < 1e-10 * abs(a), d
        assert abs(r.e1[d] - np.sum(P1 * H)) < 1e-9 * max(abs(r.e1[d]), scale)
    assert r.flops_p1 > 0 or not s.H1


@pytest.mark.parametrize("occ", ["none", "all"])
def test_dense_trivial_occupations(occ):
    s = W.config_system("chain64", n=8)
    H, _ = dense_inputs(s)
    N = H.shape[0]
    s.n_occ = 0 if occ == "none" else N
    r = T.dense_response(s, export=True)
    assert r.status == 0 and r.gap == 0.0
    want = np.zeros((N, N)) if occ == "none" else np.eye(N)
    assert np.array_equal(r.P0, want)
    assert all(np.array_equal(p, np.zeros((N, N))) for p in r.P1)
    assert r.alpha == [0.0] * len(s.H1)
    assert r.e0 == pytest.approx(0.0 if occ == "none" else np.trace(H), abs=1e-12)


def test_dense_degenerate_gap_is_an_error():
    # H = I: every eigenvalue is 1, so no gap separates the occupied states
    nb, b = 4, 2
    rp = np.arange(nb + 1, dtype=np.int64)
    ci = np.arange(nb, dtype=np.int32)
    H = W.BSR(nb, b, rp, ci, np.tile(np.eye(b), (nb, 1, 1)))
    s = W.System(H=H, H1=[], n_occ=3, xyz=np.zeros((nb, 3)))
    with pytest.raises(T.TC2Error) as ex:
        T.dense_response(s)
    assert ex.value.status == -5


def test_dense_on_a_caller_stream():
    import torch
    s = W.config_system("chain64", n=16)
    a = T.dense_response(s, export=True)
    st = torch.cuda.Stream()
    b = T.dense_response(s, export=True, stream=st.cuda_stream)
    assert np.array_equal(a.P0, b.P0) and np.array_equal(a.P1[0], b.P1[0])
    assert a.alpha == b.alpha


def test_linear_scaling_path_converges_to_the_dense_result():
    # TC2 / TC2-CPSCF with a small drop threshold against diagonalisation,
    # both on the GPU
    s = W.config_system("cube10", L=5, eps=1e-9)
    g = T.solve(s, precision="fp64")[0]
    r = T.dense_response(s, export=True)
    dx0 = np.abs(T.bsr_dense(g.X0) - r.P0).max()
    dx1 = np.abs(T.bsr_dense(g.X1[0]) - r.P1[0]).max()
    dal = abs(g.alpha[0] - r.alpha[0]) / abs(r.alpha[0])
    print(f"  TC2 vs dense: max|dX0| {dx0:.2e} max|dX1| {dx1:.2e} rel|dalpha| {dal:.2e}",
          flush=True)
    assert g.status >= 0
    assert dx0 < 1e-7 and dx1 < 1e-6 and dal < 1e-7


def test_dense_cube10_traces():
    # the benchmark system at full size (N = 13000): P0 holds n_occ states and
    # the polarizability trace is close to that of the linear-scaling solve
    s = W.config_system("cube10")
    r = T.dense_response(s)
    g = T.solve(s, precision="fp64", skip="bound", graph=True, export=False)[0]
    dal = abs(g.alpha[0] - r.alpha[0]) / abs(r.alpha[0])
    print(f"  cube10 dense: {r.seconds:.2f} s (eigh {r.ms_eigh:.0f} ms, P1 {r.ms_p1:.0f} ms); "
          f"TC2 {g.seconds:.3f} s; rel|dalpha| {dal:.2e}", flush=True)
    assert r.status == 0 and r.gap > 0
    assert abs(r.tr_p0 - s.n_occ) < 1e-8 * s.n_occ
    assert r.alpha[0] < 0
    assert dal < 1e-4
