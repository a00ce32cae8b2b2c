"""Loewdin orthogonalisation on the GPU (tc2_lowdin, tc2_congruence) against
the oracle (oracle/lowdin.py): the Newton-Schulz inverse square root, the
orthogonal forms of H and H1, the back-transform, and the whole
non-orthogonal pipeline (Loewdin -> TC2 / TC2-CPSCF -> back-transform) against
the generalised eigenproblem."""
import numpy as np
import pytest
import scipy.linalg

from oracle import exact as E
from oracle import lowdin as L
from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def dense(m):
    return O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val)


def block_pattern(X, b):
    nb = X.shape[0] // b
    blocks = X.reshape(nb, b, nb, b)
    return np.abs(blocks).sum(axis=(1, 3)) > 0


CASES = {
    "chain": lambda: W.config_system("chain64", n=12),
    "ragged_b5": lambda: W.config_system("chain64", n=11, b=5),
    "cube_b13": lambda: W.config_system("cube10", L=4),
    "three_dirs": lambda: W.config_system("cube20", L=3),
    "b16": lambda: W.config_system("chain64", n=9, b=16, occ=6),
    "b2": lambda: W.config_system("chain64", n=9, b=2, occ=1),
}


@pytest.mark.parametrize("eps", [0.0, 1e-6])
@pytest.mark.parametrize("case", list(CASES))
def test_lowdin_matches_oracle(case, eps):
    s = CASES[case]()
    S = W.make_overlap(s, amp=0.2)
    b = s.H.b
    # to a tolerance, and to a fixed number of updates
    tol, max_iter, want_status = (1e-10, 40, 0) if eps == 0.0 else (1e-14, 3, 1)
    g = T.lowdin(S, s.H, s.H1, eps=eps, tol=tol, max_iter=max_iter)
    o = L.lowdin(dense(S), dense(s.H), [dense(h) for h in s.H1], b, eps, tol, max_iter)
    print(f"  {case} eps={eps}: iters {g.iters} (oracle {o.iters}) resid {g.resid:.2e} "
          f"Z blocks {g.Z.row_ptr[-1]} {g.seconds * 1e3:.1f} ms", flush=True)
    assert g.status == want_status and o.status == want_status
    assert g.iters == o.iters
    assert abs(g.lam - o.lam) <= 1e-14 * o.lam
    assert abs(g.resid - o.resid) <= 1e-9 * o.resid + 1e-13
    for got, want in [(g.Z, o.Z), (g.H, o.H)] + list(zip(g.H1, o.H1)):
        Gd = dense(got)
        assert np.array_equal(Gd, Gd.T)                       # exactly symmetric
        assert np.array_equal(block_pattern(Gd, b), block_pattern(want, b))
        assert np.abs(Gd - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_identity_overlap_is_a_no_op():
    s = W.config_system("chain64", n=10)
    nb, b = s.H.nb, s.H.b
    S = W.BSR(nb, b, np.arange(nb + 1, dtype=np.int64), np.arange(nb, dtype=np.int32),
              np.tile(np.eye(b), (nb, 1, 1)))
    g = T.lowdin(S, s.H, s.H1, eps=1e-8)
    assert g.status == 0 and g.iters == 0 and g.resid == 0.0
    assert np.array_equal(dense(g.Z), np.eye(nb * b))
    assert np.array_equal(dense(g.H), dense(s.H))


def test_filter_floor_stops_the_iteration():
    s = W.config_system("cube10", L=3)
    S = W.make_overlap(s, amp=0.2)
    g = T.lowdin(S, s.H, [], eps=1e-3, tol=1e-14, max_iter=50)
    o = L.newton_schulz_inv_sqrt(dense(S), s.H.b, 1e-3, 1e-14, 50)
    assert g.status == 2 and o.status == 2 and g.iters == o.iters
    assert abs(g.resid - o.resid) <= 1e-9 * o.resid
    assert np.abs(dense(g.Z) - o.Z).max() < 1e-12


def test_iteration_limit():
    s = W.config_system("cube10", L=3)
    S = W.make_overlap(s, amp=0.2)
    g = T.lowdin(S, s.H, [], eps=1e-6, tol=1e-12, max_iter=1)
    assert g.status == 1 and g.iters == 1
    o = L.newton_schulz_inv_sqrt(dense(S), s.H.b, 1e-6, 1e-12, 1)
    assert np.abs(dense(g.Z) - o.Z).max() < 1e-12


def test_congruence_matches_oracle():
    s = W.config_system("cube10", L=4)
    S = W.make_overlap(s, amp=0.2)
    g = T.lowdin(S, s.H, [], eps=1e-7)
    X = s.H                                       # any symmetric block-sparse matrix
    got = dense(T.congruence(g.Z, X, eps=1e-7))
    want = L.congruence(dense(g.Z), dense(X), s.H.b, 1e-7)
    assert np.array_equal(got, got.T)
    assert np.array_equal(block_pattern(got, s.H.b), block_pattern(want, s.H.b))
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_non_orthogonal_pipeline_reaches_the_generalised_solution():
    # Loewdin -> TC2 / TC2-CPSCF on the orthogonal forms -> back-transform,
    # all on the GPU, against the generalised eigenproblem H C = S C E
    s = W.config_system("cube10", L=4, eps=1e-10)
    S = W.make_overlap(s, amp=0.2)
    eps = 1e-10
    g = T.lowdin(S, s.H, s.H1, eps=eps, tol=1e-9, max_iter=20)
    orth = W.System(H=g.H, H1=g.H1, n_occ=s.n_occ, xyz=s.xyz, eps=eps, tol=1e-11)
    r = T.solve(orth, precision="fp64")[0]
    assert r.status >= 0
    P0 = dense(T.congruence(g.Z, r.X0, eps=eps))
    P1 = dense(T.congruence(g.Z, r.X1[0], eps=eps))
    H, Sd, H1 = dense(s.H), dense(S), dense(s.H1[0])
    e, C = scipy.linalg.eigh(H, Sd)
    Co = C[:, :s.n_occ]
    P0_ref = Co @ Co.T
    # P1 of the generalised problem for a perturbation of H alone (S fixed):
    # Z_exact times the orthogonal response times Z_exact
    ev, V = np.linalg.eigh(Sd)
    Ze = (V / np.sqrt(ev)) @ V.T
    P1_ref = Ze @ E.exact_response(Ze @ H @ Ze, Ze @ H1 @ Ze, s.n_occ) @ Ze
    a_ref = float(np.sum(P1_ref * H1))
    d0, d1 = np.abs(P0 - P0_ref).max(), np.abs(P1 - P1_ref).max()
    da = abs(r.alpha[0] - a_ref) / abs(a_ref)
    print(f"  non-orthogonal: max|dP0| {d0:.2e} max|dP1| {d1:.2e} rel|dalpha| {da:.2e} "
          f"(NS {g.iters} updates, TC2 {r.iters} updates)", flush=True)
    assert d0 < 1e-7 and d1 < 1e-6 and da < 1e-8
    np.testing.assert_allclose(P0 @ Sd @ P0, P0, atol=1e-7)        # P S P = P
    assert abs(np.trace(P0 @ Sd) - s.n_occ) < 1e-6


def test_lowdin_cube10_full_size():
    # the benchmark system (N = 13000) with a synthetic overlap: quadratic
    # convergence to tol, an exactly symmetric S^-1/2, and Z S Z = I on a
    # sample of block rows
    s = W.config_system("cube10")
    S = W.make_overlap(s, amp=0.2)
    g = T.lowdin(S, s.H, s.H1, eps=1e-6, tol=1e-9, max_iter=40)
    print(f"  cube10: status {g.status} {g.iters} updates, resid {g.resid:.2e}, {g.seconds:.2f} s, "
          f"Z blocks {g.Z.row_ptr[-1]}, H_orth blocks {g.H.row_ptr[-1]}", flush=True)
    assert g.status in (0, 2) and g.iters <= 15 and g.resid < 1e-5
    Z = g.Z
    b, nb = Z.b, Z.nb
    rows = np.random.default_rng(0).choice(nb, size=12, replace=False)
    Sd = {}
    for I in range(nb):
        for p in range(int(S.row_ptr[I]), int(S.row_ptr[I + 1])):
            Sd[(I, int(S.col[p]))] = S.val[p]
    Zb = {}
    for I in range(nb):
        for p in range(int(Z.row_ptr[I]), int(Z.row_ptr[I + 1])):
            Zb[(I, int(Z.col[p]))] = Z.val[p]
    zrow = lambda I: {J: Zb[(I, J)] for J in Z.col[Z.row_ptr[I]:Z.row_ptr[I + 1]]}
    for I in rows:
        # row I of Z S Z, dense over block columns
        zs = {}
        for K, zik in zrow(int(I)).items():
            for p in range(int(S.row_ptr[K]), int(S.row_ptr[K + 1])):
                L_ = int(S.col[p])
                zs[L_] = zs.get(L_, 0.0) + zik @ S.val[p]
        out = {}
        for L_, m in zs.items():
            for J, zlj in zrow(L_).items():
                out[J] = out.get(J, 0.0) + m @ zlj
        for J, blk in out.items():
            want = np.eye(b) if J == I else np.zeros((b, b))
            assert np.abs(blk - want).max() < 1e-4, (I, J)


# ---------------------------------------------------------------- moving overlap (displacements)
def displaced(case):
    s = CASES[case]()
    S = W.make_overlap(s, amp=0.2)
    H1, S1 = W.make_displacement(s, atom=s.H.nb // 2)
    return s, S, H1, S1


@pytest.mark.parametrize("eps", [0.0, 1e-6])
@pytest.mark.parametrize("case", ["chain", "ragged_b5", "cube_b13"])
def test_lowdin_response_matches_oracle(case, eps):
    s, S, H1, S1 = displaced(case)
    b = s.H.b
    tol, max_iter, want_status = (1e-10, 40, 0) if eps == 0.0 else (1e-14, 3, 1)
    g = T.lowdin_response(S, s.H, [H1], [S1], eps=eps, tol=tol, max_iter=max_iter)
    o = L.lowdin_response(dense(S), [dense(S1)], dense(s.H), [dense(H1)], b, eps, tol, max_iter)
    print(f"  {case} eps={eps}: iters {g.iters} Z1 blocks {g.Z1[0].row_ptr[-1]} "
          f"H1_orth blocks {g.H1[0].row_ptr[-1]} {g.seconds * 1e3:.1f} ms", flush=True)
    assert g.status == want_status and o.status == want_status and g.iters == o.iters
    for got, want in [(g.Z, o.Z), (g.H, o.H), (g.Z1[0], o.Z1[0]), (g.H1[0], o.H1[0])]:
        Gd = dense(got)
        assert np.array_equal(Gd, Gd.T)
        assert np.array_equal(block_pattern(Gd, b), block_pattern(want, b))
        assert np.abs(Gd - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_field_case_of_the_response_entry_is_unchanged():
    # S1 = 0: the same Z and H1_orth as tc2_lowdin, and Z1 = 0
    s, S, H1, S1 = displaced("chain")
    z = W.BSR(S1.nb, S1.b, np.zeros(S1.nb + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
              np.zeros((0, S1.b, S1.b)))
    g = T.lowdin_response(S, s.H, [H1], [z], eps=1e-6)
    f = T.lowdin(S, s.H, [H1], eps=1e-6)
    assert g.Z1[0].row_ptr[-1] == 0
    assert np.array_equal(dense(g.Z), dense(f.Z)) and np.array_equal(dense(g.H1[0]), dense(f.H1[0]))


def test_congruence_response_matches_oracle():
    s, S, H1, S1 = displaced("cube_b13")
    g = T.lowdin_response(S, s.H, [H1], [S1], eps=1e-7)
    X, X1 = s.H, H1                                  # any symmetric pair
    got = dense(T.congruence_response(g.Z, g.Z1[0], X, X1, eps=1e-7))
    want = L.congruence_response(dense(g.Z), dense(g.Z1[0]), dense(X), dense(X1), s.H.b, 1e-7)
    assert np.array_equal(got, got.T)
    assert np.array_equal(block_pattern(got, s.H.b), block_pattern(want, s.H.b))
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_displacement_pipeline_reaches_the_generalised_response():
    # Loewdin with the overlap derivative -> TC2 / TC2-CPSCF on H_orth and
    # H1_orth -> three-term back-transform, all on the GPU, against finite
    # differences of the projector of H C = S C E when H and S both move
    s, S, H1, S1 = displaced("cube_b13")
    eps = 1e-10
    g = T.lowdin_response(S, s.H, [H1], [S1], eps=eps, tol=1e-9, max_iter=20)
    orth = W.System(H=g.H, H1=g.H1, n_occ=s.n_occ, xyz=s.xyz, eps=eps, tol=1e-11)
    r = T.solve(orth, precision="fp64")[0]
    assert r.status >= 0
    P1 = dense(T.congruence_response(g.Z, g.Z1[0], r.X0, r.X1[0], eps=eps))
    H, Sd, H1d, S1d = dense(s.H), dense(S), dense(H1), dense(S1)

    def proj(x):
        e, C = scipy.linalg.eigh(H + x * H1d, Sd + x * S1d)
        Co = C[:, :s.n_occ]
        return Co @ Co.T
    h = 1e-5
    fd = (proj(h) - proj(-h)) / (2 * h)
    d1 = np.abs(P1 - fd).max()
    print(f"  displacement: max|dP1| {d1:.2e} (max|P1| {np.abs(fd).max():.2e}; NS {g.iters}, "
          f"TC2 {r.iters} updates)", flush=True)
    assert np.abs(fd).max() > 1e-3
    assert d1 < 1e-6
