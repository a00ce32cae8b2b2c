"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, hand-worked steps, invariants, limits), not against itself."""
import numpy as np
import pytest

from oracle import tc2_oracle as O
from oracle import exact as E
from paper_2009_03551_amd import workloads as W


def dense(bsr):
    return O.bsr_to_dense(bsr.nb, bsr.b, bsr.row_ptr, bsr.col, bsr.val)


# ---------------------------------------------------------------- Gershgorin
def test_gershgorin_hand_2x2():
    # discs: 1 +- 2 and 3 +- 2  ->  [-1, 5]
    assert O.gershgorin(np.array([[1.0, -2.0], [-2.0, 3.0]])) == (-1.0, 5.0)


def test_gershgorin_hand_3x3():
    H = np.array([[2.0, 0.5, 0.0], [0.5, -1.0, 0.25], [0.0, 0.25, 4.0]])
    # rows: 2 +- 0.5, -1 +- 0.75, 4 +- 0.25
    assert O.gershgorin(H) == (-1.75, 4.25)


def test_gershgorin_diagonal_is_exact():
    H = np.diag([3.0, -2.5, 0.5])
    assert O.gershgorin(H) == (-2.5, 3.0)


def test_gershgorin_contains_spectrum():
    s = W.config_system("chain64", n=12)
    H = dense(s.H)
    lo, hi = O.gershgorin(H)
    ev = np.linalg.eigvalsh(H)
    assert lo <= ev[0] and hi >= ev[-1]


# ---------------------------------------------------------------- init
def test_init_maps_spectrum_reversed_into_unit_interval():
    s = W.config_system("chain64", n=10)
    H = dense(s.H)
    lo, hi = O.gershgorin(H)
    X0, X1 = O.tc2_init(H, [dense(s.H1[0])], lo, hi)
    ev = np.linalg.eigvalsh(H)
    ex = np.linalg.eigvalsh(X0)
    np.testing.assert_allclose(np.sort((hi - ev) / (hi - lo)), ex, atol=1e-14)
    assert ex[0] >= -1e-15 and ex[-1] <= 1 + 1e-15
    np.testing.assert_allclose(X1[0], -dense(s.H1[0]) / (hi - lo), rtol=0, atol=0)


# ---------------------------------------------------------------- one step by hand
def test_step_square_hand():
    X0 = np.diag([0.2, 0.9])
    X1 = np.array([[0.0, 0.5], [0.5, 0.0]])
    A, B = O.tc2_step(X0, [X1], square=True)
    np.testing.assert_allclose(A, np.diag([0.04, 0.81]), atol=1e-15)
    # X1 X0 + X0 X1 = 0.5 * (0.2 + 0.9) off the diagonal
    np.testing.assert_allclose(B[0], [[0.0, 0.55], [0.55, 0.0]], atol=1e-15)


def test_step_double_hand():
    X0 = np.diag([0.2, 0.9])
    X1 = np.array([[0.0, 0.5], [0.5, 0.0]])
    A, B = O.tc2_step(X0, [X1], square=False)
    np.testing.assert_allclose(A, np.diag([0.36, 0.99]), atol=1e-15)
    np.testing.assert_allclose(B[0], [[0.0, 0.45], [0.45, 0.0]], atol=1e-15)


def test_step_response_non_commuting_hand():
    # X0 = [[1,1],[1,0]]/2, X1 = [[1,0],[0,-1]]: X1 X0 + X0 X1 = [[1,0],[0,0]]
    X0 = np.array([[0.5, 0.5], [0.5, 0.0]])
    X1 = np.array([[1.0, 0.0], [0.0, -1.0]])
    _, B = O.tc2_step(X0, [X1], square=True)
    np.testing.assert_allclose(B[0], [[1.0, 0.0], [0.0, 0.0]], atol=1e-15)
    _, B = O.tc2_step(X0, [X1], square=False)
    np.testing.assert_allclose(B[0], [[1.0, 0.0], [0.0, -2.0]], atol=1e-15)


# ---------------------------------------------------------------- block filter
def test_block_drop_hand():
    b, eps = 2, 1e-3
    X = np.zeros((6, 6))
    X[0:2, 0:2] = [[1e-9, 0.0], [0.0, 0.0]]      # diagonal block: never dropped
    X[0:2, 2:4] = [[2e-3, 0.0], [0.0, 0.0]]      # norm 2e-3: kept
    X[0:2, 4:6] = [[3e-4, 0.0], [0.0, 4e-4]]     # norm 5e-4: dropped
    X[2:4, 4:6] = [[0.0, 9.9e-4], [0.0, 0.0]]    # norm 9.9e-4: dropped
    X = X + np.triu(X, 2).T                      # mirror the off-diagonal blocks
    Y = O.block_drop(X, b, eps)
    Z = np.zeros((6, 6))
    Z[0:2, 0:2] = [[1e-9, 0.0], [0.0, 0.0]]
    Z[0:2, 2:4] = [[2e-3, 0.0], [0.0, 0.0]]
    Z[2:4, 0:2] = [[2e-3, 0.0], [0.0, 0.0]]
    assert np.array_equal(Y, Z)
    assert np.array_equal(O.block_drop(X, b, 0.0), X)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("delta,t", [(0.3, 0.4), (1.0, 0.05), (-0.2, 0.7)])
def test_dimer_closed_form(delta, t):
    # H = [[-D, t], [t, D]], H1 = diag(-1/2, 1/2), one occupied state.
    # With E = sqrt(D^2 + t^2): P0 = (I - H/E)/2 and
    # Tr(P1 H1) = -t^2 / (4 E^3)  (first-order perturbation of the projector).
    H = np.array([[-delta, t], [t, delta]])
    H1 = np.diag([-0.5, 0.5])
    Eg = np.hypot(delta, t)
    r = O.tc2_solve(H, [H1], 1, 1, eps=0.0, tol=1e-14, max_iter=200)
    np.testing.assert_allclose(r.X0, (np.eye(2) - H / Eg) / 2, atol=1e-12)
    assert abs(r.alpha[0] - (-t * t / (4 * Eg ** 3))) < 1e-11
    P1 = -0.5 * (H1 / Eg - H * delta / (2 * Eg ** 3))
    np.testing.assert_allclose(r.X1[0], P1, atol=1e-11)


def test_limit_is_projector_and_sum_over_states():
    s = W.config_system("chain64", n=24)
    H, H1 = dense(s.H), dense(s.H1[0])
    r = O.tc2_solve(H, [H1], s.n_occ, s.H.b, eps=0.0, tol=1e-13)
    assert r.status == O.STATUS_OK
    np.testing.assert_allclose(r.X0, E.exact_projector(H, s.n_occ), atol=1e-12)
    np.testing.assert_allclose(r.X1[0], E.exact_response(H, H1, s.n_occ), atol=1e-11)
    assert abs(r.alpha[0] - E.exact_alpha(H, H1, s.n_occ)) < 1e-10 * abs(r.alpha[0])


def test_exact_response_is_derivative_of_projector():
    # pins the closed form itself: central difference of the eigh projector
    s = W.config_system("chain64", n=10)
    H, H1 = dense(s.H), dense(s.H1[0])
    h = 1e-5
    fd = (E.exact_projector(H + h * H1, s.n_occ) - E.exact_projector(H - h * H1, s.n_occ)) / (2 * h)
    np.testing.assert_allclose(E.exact_response(H, H1, s.n_occ), fd, atol=1e-8)
    assert abs(E.exact_alpha(H, H1, s.n_occ) - np.sum(fd * H1)) < 1e-7


def test_response_recursion_is_derivative_of_tc2_map():
    # With the branch sequence and the spectral bounds held fixed, X1_n must be
    # the derivative of X0_n along H1 (the recursion differentiates Eq. TC2).
    s = W.config_system("chain64", n=8)
    H, H1 = dense(s.H), dense(s.H1[0])
    lo, hi = O.gershgorin(H)
    ref = O.tc2_solve(H, [H1], s.n_occ, s.H.b, eps=0.0, tol=1e-12)
    h = 1e-6

    def run(Hx):
        X0, X1 = O.tc2_init(Hx, [H1], lo, hi)
        for c in ref.branches:
            X0, X1 = O.tc2_step(X0, X1, c == "S")
        return X0, X1

    Xp, _ = run(H + h * H1)
    Xm, _ = run(H - h * H1)
    _, X1 = run(H)
    np.testing.assert_allclose(X1[0], (Xp - Xm) / (2 * h), atol=2e-6 * np.abs(X1[0]).max())


# ---------------------------------------------------------------- invariants at convergence
def test_invariants_with_filter():
    s = W.config_system("chain64")
    H, H1 = dense(s.H), dense(s.H1[0])
    r = O.tc2_solve(H, [H1], s.n_occ, s.H.b, eps=s.eps, tol=s.tol)
    X0, X1 = r.X0, r.X1[0]
    tol = 1e-5
    assert abs(np.trace(X0) - s.n_occ) < tol
    assert np.abs(X0 @ X0 - X0).max() < tol
    assert abs(np.trace(X1)) < tol
    assert np.abs(X0 @ X1 + X1 @ X0 - X1).max() < tol
    assert np.abs(H @ X0 - X0 @ H).max() < tol
    assert np.abs(H @ X1 - X1 @ H + H1 @ X0 - X0 @ H1).max() < tol
    assert abs(np.sum(X1 * H)) < tol
    # the filter keeps the result near the exact limit (error ~ eps)
    assert np.abs(X1 - E.exact_response(H, H1, s.n_occ)).max() < 20 * s.eps
    # iteration count of the order the paper reports (about 25 cycles)
    assert 12 <= r.iters <= 30


def test_decoupled_atoms_give_onsite_projector():
    # No off-site coupling: the projector is block diagonal, each block the
    # projector of its own onsite block; a field that is constant on each atom
    # commutes with H, so the response vanishes.  The onsite blocks are rotated
    # so that the Gershgorin bounds are not tight.
    rng = np.random.default_rng(11)
    b, nb = 8, 6
    n = b * nb
    H = np.zeros((n, n))
    P = np.zeros((n, n))
    for I in range(nb):
        Q, _ = np.linalg.qr(rng.standard_normal((b, b)))
        e = np.concatenate([-1 + 0.1 * rng.random(4), 1 + 0.1 * rng.random(4)])
        H[I * b:(I + 1) * b, I * b:(I + 1) * b] = (Q * e) @ Q.T
        P[I * b:(I + 1) * b, I * b:(I + 1) * b] = Q[:, :4] @ Q[:, :4].T
    H1 = np.diag(np.repeat(np.arange(nb) - 2.5, b))
    r = O.tc2_solve(H, [H1], 4 * nb, b, eps=1e-7, tol=1e-12)
    np.testing.assert_allclose(r.X0, P, atol=1e-12)
    assert np.abs(r.X1[0]).max() < 1e-10


@pytest.mark.parametrize("occ", ["none", "all"])
def test_nocc_edges(occ):
    s = W.config_system("chain64", n=4)
    H, H1 = dense(s.H), dense(s.H1[0])
    n_occ = 0 if occ == "none" else H.shape[0]
    r = O.tc2_solve(H, [H1], n_occ, s.H.b, eps=1e-7, tol=1e-9)
    assert np.array_equal(r.X0, np.zeros_like(H) if occ == "none" else np.eye(H.shape[0]))
    assert not np.any(r.X1[0])


# ---------------------------------------------------------------- metamorphic relations
def test_scale_and_shift_of_h():
    s = W.config_system("chain64", n=16)
    H, H1 = dense(s.H), dense(s.H1[0])
    a = O.tc2_solve(H, [H1], s.n_occ, 8, eps=0.0, tol=1e-12)
    sc, sh = 2.0, 0.7
    b = O.tc2_solve(sc * H + sh * np.eye(H.shape[0]), [H1], s.n_occ, 8, eps=0.0,
                    tol=1e-12, replay=a.branches)
    np.testing.assert_allclose(b.X0, a.X0, atol=1e-11)
    np.testing.assert_allclose(b.X1[0] * sc, a.X1[0], atol=1e-10)


def test_shift_of_h1_leaves_response():
    s = W.config_system("chain64", n=16)
    H, H1 = dense(s.H), dense(s.H1[0])
    a = O.tc2_solve(H, [H1], s.n_occ, 8, eps=0.0, tol=1e-13)
    b = O.tc2_solve(H, [H1 + 3.0 * np.eye(H.shape[0])], s.n_occ, 8, eps=0.0,
                    tol=1e-13, replay=a.branches)
    np.testing.assert_allclose(b.X1[0], a.X1[0], atol=1e-10)


def test_linear_in_h1():
    s = W.config_system("chain64", n=12, n_dir=2)
    H, Hx = dense(s.H), dense(s.H1[0])
    rng = np.random.default_rng(7)
    G = rng.standard_normal(H.shape)
    G = G + G.T
    a = O.tc2_solve(H, [Hx, G, 2 * Hx - 3 * G], s.n_occ, 8, eps=0.0, tol=1e-12)
    np.testing.assert_allclose(a.X1[2], 2 * a.X1[0] - 3 * a.X1[1], atol=1e-11)


def test_atom_permutation():
    s = W.config_system("chain64", n=10)
    H, H1 = dense(s.H), dense(s.H1[0])
    b = 8
    perm = np.random.default_rng(3).permutation(10)
    idx = (perm[:, None] * b + np.arange(b)[None, :]).ravel()
    a = O.tc2_solve(H, [H1], s.n_occ, b, eps=1e-6, tol=1e-10)
    c = O.tc2_solve(H[np.ix_(idx, idx)], [H1[np.ix_(idx, idx)]], s.n_occ, b,
                    eps=1e-6, tol=1e-10)
    assert a.branches == c.branches
    np.testing.assert_allclose(c.X0, a.X0[np.ix_(idx, idx)], atol=1e-12)
    np.testing.assert_allclose(c.X1[0], a.X1[0][np.ix_(idx, idx)], atol=1e-11)


def test_filter_error_grows_with_eps():
    # the filter error grows roughly linearly with the threshold (Sec. 2.3)
    s = W.config_system("chain64", n=32)
    H, H1 = dense(s.H), dense(s.H1[0])
    P1 = E.exact_response(H, H1, s.n_occ)
    errs = []
    for eps in (1e-7, 1e-6, 1e-5):
        r = O.tc2_solve(H, [H1], s.n_occ, 8, eps=eps, tol=1e-10)
        errs.append(np.abs(r.X1[0] - P1).max())
    assert errs[0] < errs[1] < errs[2]
    assert errs[2] < 100 * 1e-5


def test_replay_reproduces_run():
    s = W.config_system("chain64", n=16)
    H, H1 = dense(s.H), dense(s.H1[0])
    a = O.tc2_solve(H, [H1], s.n_occ, 8, eps=1e-7, tol=1e-9)
    b = O.tc2_solve(H, [H1], s.n_occ, 8, eps=1e-7, tol=1e-9, replay=a.branches)
    assert np.array_equal(a.X0, b.X0) and np.array_equal(a.X1[0], b.X1[0])


def test_closing_pair_branches_are_opposite():
    s = W.config_system("chain64", n=16)
    H, H1 = dense(s.H), dense(s.H1[0])
    a = O.tc2_solve(H, [H1], s.n_occ, 8, eps=1e-7, tol=1e-9)
    c = O.tc2_solve(H, [H1], s.n_occ, 8, eps=1e-7, tol=1e-9, closing_pair=True)
    assert c.branches[:-2] == a.branches
    assert c.branches[-1] != c.branches[-2]
    assert np.abs(c.X1[0] - a.X1[0]).max() < 1e-6


def test_band_energies_at_convergence():
    # E0 = Tr(P0 H) is the sum of the N_occ lowest eigenvalues; E1 = Tr(P1 H)
    # vanishes (P1 couples occupied and virtual states only); alpha is the
    # sum-over-states trace.
    s = W.config_system("chain64", n=16)
    H, H1 = dense(s.H), dense(s.H1[0])
    r = O.tc2_solve(H, [H1], s.n_occ, 8, eps=0.0, tol=1e-12, keep_history=True)
    last = r.history[-1]
    ev = np.linalg.eigvalsh(H)
    assert abs(last["E0"] - ev[:s.n_occ].sum()) < 1e-10
    assert abs(last["E1"][0]) < 1e-10
    assert abs(last["alpha"][0] - E.exact_alpha(H, H1, s.n_occ)) < 1e-9


def test_band_energies_hand():
    X0 = np.array([[1.0, 2.0], [2.0, 0.5]])
    X1 = np.array([[0.0, 1.0], [1.0, -1.0]])
    H = np.array([[3.0, -1.0], [-1.0, 2.0]])
    H1 = np.diag([0.5, -0.5])
    E0, E1, al = O.band_energies(X0, [X1], H, [H1])
    assert E0 == 3.0 - 2.0 - 2.0 + 1.0          # Tr(X0 H)
    assert E1 == [0.0 - 1.0 - 1.0 - 2.0]        # Tr(X1 H)
    assert al == [0.5]                          # Tr(X1 H1)


# ---------------------------------------------------------------- stopping rule (Sec. 2.3 tolerance, stall guard)
def _e(E0, E1, al):
    """Scalars of one iterate in the form band_energies returns."""
    return (E0, list(E1), list(al))


def test_convergence_needs_two_updates():
    # a change far below tol after the first update does not stop it: the
    # first update compares with the unfiltered initial matrices
    prev, cur = _e(1.0, [0.0], [-3.0]), _e(1.0, [0.0], [-3.0])
    assert O.stopping_rule(1, prev, cur, [0.5], 1e-9) is None
    assert O.stopping_rule(2, prev, cur, [0.5, 0.4], 1e-9) == O.STATUS_OK


def test_convergence_is_strict_and_absolute():
    tol = 1e-6
    prev = _e(-100.0, [0.25], [-7.0])
    falling = [0.5, 0.4, 0.3, 0.2, 0.1]   # the stall guard stays quiet
    assert O.stopping_rule(5, prev, _e(-100.0 + 0.5e-6, [0.25], [-7.0]), falling, tol) == O.STATUS_OK
    # |dE0| == tol (exactly representable) is not below tol
    assert O.stopping_rule(5, prev, _e(-100.0 + 2.0 ** -20, [0.25], [-7.0]), falling,
                           2.0 ** -20) is None


def test_alpha_change_alone_blocks_convergence():
    # E0 and Tr(X1 H) unchanged, the polarizability trace still moving
    tol = 1e-9
    prev = _e(-12.5, [1e-12], [-40.0])
    cur = _e(-12.5, [1e-12], [-40.0 + 3e-9])
    assert O.stopping_rule(6, prev, cur, [0.9, 0.8, 0.7, 0.6, 0.5, 0.4], tol) is None
    # ... and only alpha: the same change in a second direction's alpha
    prev2 = _e(-12.5, [0.0, 0.0], [-40.0, -41.0])
    cur2 = _e(-12.5, [0.0, 0.0], [-40.0, -41.0 - 2e-9])
    assert O.stopping_rule(6, prev2, cur2, [0.9, 0.8, 0.7, 0.6, 0.5, 0.4], tol) is None
    # a change of E1_d alone blocks it too
    cur3 = _e(-12.5, [0.0, 5e-9], [-40.0, -41.0])
    assert O.stopping_rule(6, prev2, cur3, [0.9, 0.8, 0.7, 0.6, 0.5, 0.4], tol) is None


def _guard(iotas):
    """Stall-guard decision after the last of ``iotas``, with energies that
    keep moving (so the convergence test cannot stop it)."""
    k = len(iotas)
    return O.stopping_rule(k, _e(0.0, [], []), _e(1.0, [], []), iotas, 1e-9)


def test_stall_guard_compares_with_two_updates_back():
    # |iota_3| >= |iota_1| while |iota_3| < |iota_2|: fires (k-2), where a
    # comparison with k-1 would not
    assert _guard([0.3, 0.6, 0.4]) == O.STATUS_FLOOR
    # |iota_3| < |iota_1| while |iota_3| >= |iota_2|: does not fire, where a
    # comparison with k-1 would
    assert _guard([0.5, 0.3, 0.4]) is None
    # equality fires (>=); signs do not matter (absolute values)
    assert _guard([0.5, 0.1, -0.5]) == O.STATUS_FLOOR


def test_stall_guard_needs_small_iota_and_three_updates():
    # |iota| >= 1: far from idempotent, no floor yet
    assert _guard([2.0, 1.5, 2.5]) is None
    assert _guard([1.0, 0.5, 1.0]) is None
    # fewer than three updates: nothing two updates back
    assert _guard([0.3, 0.6]) is None
    # a later index uses the right pair: iota_5 against iota_3 only
    assert _guard([0.01, 0.9, 0.2, 0.1, 0.15]) is None     # 0.15 < 0.2
    assert _guard([0.9, 0.01, 0.2, 0.1, 0.25]) == O.STATUS_FLOOR


def test_convergence_is_tested_before_the_guard():
    # both would stop: the tolerance test decides (status OK)
    prev = cur = _e(0.5, [0.0], [-1.0])
    assert O.stopping_rule(3, prev, cur, [0.3, 0.6, 0.4], 1e-9) == O.STATUS_OK


def test_solve_stops_where_the_rule_first_fires():
    # with an unreachable tolerance the guard alone stops the solve: at the
    # first update k >= 3 with |iota_k| < 1 and |iota_k| >= |iota_{k-2}|
    s = W.config_system("chain64", n=24)
    r = O.solve_system(s, tol=1e-300, keep_history=True, max_iter=80)
    io = [abs(h["iota"]) for h in r.history]
    first = next(k for k in range(3, len(io) + 1)
                 if io[k - 1] < 1.0 and io[k - 1] >= io[k - 3])
    assert r.status == O.STATUS_FLOOR
    assert r.iters == first == len(io) == 23
    # on this run a guard comparing with k-1 would stop one update earlier
    k1 = next(k for k in range(3, len(io) + 1) if io[k - 1] < 1.0 and io[k - 1] >= io[k - 2])
    assert k1 == 22


# ---------------------------------------------------------------- useful block products of an update
def _brute_useful(prev, new, b):
    """The same count by a triple loop over block indices (the definition
    written out element by element)."""
    nb = prev[0].shape[0] // b
    nz = lambda X, i, j: np.any(X[i * b:(i + 1) * b, j * b:(j + 1) * b] != 0.0)
    total = 0
    for I in range(nb):
        for J in range(I, nb):
            for K in range(nb):
                if nz(new[0], I, J) and nz(prev[0], I, K) and nz(prev[0], K, J):
                    total += 1
                for d in range(1, len(prev)):
                    if nz(new[d], I, J):
                        total += int(nz(prev[0], I, K) and nz(prev[d], K, J))
                        total += int(nz(prev[d], I, K) and nz(prev[0], K, J))
    return total


def test_useful_products_by_hand():
    # 3 blocks of size 1; X0 tridiagonal, X1 diagonal; after the update every
    # X0 block is kept, X1 keeps only (0, 0) and (0, 1)
    X0 = np.array([[1.0, 0.5, 0.0], [0.5, 1.0, 0.5], [0.0, 0.5, 1.0]])
    X1 = np.diag([0.2, 0.0, 0.3])
    N0 = np.ones((3, 3))
    N1 = np.zeros((3, 3))
    N1[0, 0] = N1[0, 1] = N1[1, 0] = 1.0
    # X0 X0 on upper outputs: (0,0): K=0,1 -> 2; (0,1): K=0,1 -> 2; (0,2): K=1 -> 1;
    # (1,1): 3; (1,2): 2; (2,2): 2  => 12
    # X0 X1 + X1 X0 at (0,0): X0_00 X1_00 + X1_00 X0_00 = 2; at (0,1): X0_0K X1_K1 (X1_11 = 0) -> 0,
    # X1_0K X0_K1: K = 0 -> 1  => 3
    assert O.useful_products([X0, X1], [N0, N1], 1) == 15
    assert _brute_useful([X0, X1], [N0, N1], 1) == 15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_useful_products_equals_the_triple_loop(seed):
    rng = np.random.default_rng(seed)
    nb, b, D = 7, 2, 2

    def sym_blocks(p):
        m = np.triu(rng.random((nb, nb)) < p)
        m = m | m.T | np.eye(nb, dtype=bool)
        X = rng.standard_normal((nb * b, nb * b)) * np.kron(m, np.ones((b, b)))
        return X + X.T
    prev = [sym_blocks(0.4) for _ in range(1 + D)]
    new = [sym_blocks(0.6) for _ in range(1 + D)]
    prev[1][:b, :] = 0.0                        # an empty block row of X1_1
    assert O.useful_products(prev, new, b) == _brute_useful(prev, new, b)
