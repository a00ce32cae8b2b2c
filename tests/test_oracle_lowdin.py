"""Pins of the Loewdin oracle (oracle/lowdin.py) against what linear algebra
fixes independently of it: S^-1/2 from an eigendecomposition, the
generalised eigenproblem H C = S C E (scipy), the non-orthogonal idempotency
P S P = P, and finite differences of the generalised projector."""
import numpy as np
import pytest
import scipy.linalg

from oracle import exact as E
from oracle import lowdin as L
from oracle import tc2_oracle as O
from paper_2009_03551_amd import workloads as W


def dense(m):
    return O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val)


def problem(name="chain", amp=0.2):
    s = W.config_system("chain64", n=8) if name == "chain" else W.config_system("cube10", L=3)
    S = dense(W.make_overlap(s, amp=amp))
    return s, S, dense(s.H), [dense(h) for h in s.H1]


def inv_sqrt(S):
    e, V = np.linalg.eigh(S)
    return (V / np.sqrt(e)) @ V.T


def generalised_projector(H, S, n_occ):
    e, C = scipy.linalg.eigh(H, S)          # C^T S C = I
    Co = C[:, :n_occ]
    return Co @ Co.T


@pytest.mark.parametrize("name", ["chain", "cube"])
def test_newton_schulz_reaches_the_inverse_square_root(name):
    s, S, _, _ = problem(name)
    r = L.newton_schulz_inv_sqrt(S, s.H.b, 0.0, 1e-14, 50)
    assert r.status == L.STATUS_OK and 3 <= r.iters <= 30
    np.testing.assert_allclose(r.Z, inv_sqrt(S), atol=1e-12)
    np.testing.assert_allclose(r.Z @ S @ r.Z, np.eye(S.shape[0]), atol=1e-12)
    lam = np.linalg.eigvalsh(S).max()
    assert lam <= r.lam * (1 + 1e-12)                 # Gershgorin bound is an upper bound


def test_orthogonal_form_has_the_generalised_spectrum():
    s, S, H, H1 = problem("cube")
    o = L.lowdin(S, H, H1, s.H.b, 0.0, 1e-14, 50)
    want = scipy.linalg.eigh(H, S, eigvals_only=True)
    np.testing.assert_allclose(np.linalg.eigvalsh(o.H), want, atol=1e-11)
    assert np.array_equal(o.H, o.H.T)


def test_back_transform_gives_the_non_orthogonal_density_matrix():
    s, S, H, H1 = problem("chain")
    o = L.lowdin(S, H, H1, s.H.b, 0.0, 1e-14, 50)
    P0 = L.congruence(o.Z, E.exact_projector(o.H, s.n_occ), s.H.b, 0.0)
    np.testing.assert_allclose(P0, generalised_projector(H, S, s.n_occ), atol=1e-11)
    np.testing.assert_allclose(P0 @ S @ P0, P0, atol=1e-11)       # P S P = P
    assert abs(np.trace(P0 @ S) - s.n_occ) < 1e-10


def test_back_transformed_response_is_the_derivative_of_the_projector():
    # S fixed (a field perturbation): P1 = Z P1_orth Z with P1_orth from H1_orth
    s, S, H, H1 = problem("chain")
    o = L.lowdin(S, H, H1, s.H.b, 0.0, 1e-14, 50)
    P1 = L.congruence(o.Z, E.exact_response(o.H, o.H1[0], s.n_occ), s.H.b, 0.0)
    h = 1e-5
    fd = (generalised_projector(H + h * H1[0], S, s.n_occ)
          - generalised_projector(H - h * H1[0], S, s.n_occ)) / (2 * h)
    np.testing.assert_allclose(P1, fd, atol=1e-7)


def test_filtered_iteration_stays_near_the_exact_root_and_symmetric():
    s, S, H, H1 = problem("cube")
    eps = 1e-6
    r = L.newton_schulz_inv_sqrt(S, s.H.b, eps, 1e-9, 50)
    assert r.status == L.STATUS_OK
    assert np.array_equal(r.Z, r.Z.T)
    assert np.abs(r.Z - inv_sqrt(S)).max() < 100 * eps
    # dropped blocks are whole blocks
    nb, b = s.H.nb, s.H.b
    blocks = r.Z.reshape(nb, b, nb, b)
    norms = np.sqrt(np.einsum("iajb,iajb->ij", blocks, blocks))
    assert np.all((norms == 0) | (norms >= eps / np.sqrt(r.lam) * 0.999) | np.eye(nb, dtype=bool))


def test_products_follow_their_definitions():
    rng = np.random.default_rng(3)
    b, nb = 3, 4
    A = rng.standard_normal((nb * b, nb * b))
    A = A + A.T
    B = rng.standard_normal((nb * b, nb * b))
    B = B + B.T
    C = L.symmetric_product(A, B, b, 0.0)
    assert np.array_equal(C, C.T)
    full = A @ B
    for I in range(nb):
        for J in range(I, nb):
            blk = C[I * b:(I + 1) * b, J * b:(J + 1) * b]
            ref = full[I * b:(I + 1) * b, J * b:(J + 1) * b]
            if I < J:
                assert np.array_equal(blk, ref)
            else:
                assert np.array_equal(np.triu(blk), np.triu(ref))
    # the plain product drops each off-diagonal block on its own
    big = L.product(A, B, b, np.inf)
    assert np.array_equal(big, full * np.kron(np.eye(nb), np.ones((b, b))))


def test_filter_floor_stops_the_iteration():
    # with a coarse filter the residual levels off above a tiny tolerance
    s, S, _, _ = problem("cube")
    r = L.newton_schulz_inv_sqrt(S, s.H.b, 1e-3, 1e-14, 50)
    assert r.status == L.STATUS_FLOOR and r.iters < 15
    assert r.resid > 1e-10
    # without it, quadratic convergence reaches the tolerance first
    r0 = L.newton_schulz_inv_sqrt(S, s.H.b, 0.0, 1e-12, 50)
    assert r0.status == L.STATUS_OK and r0.iters < r.iters + 3


def test_iteration_limit_reports_not_converged():
    s, S, _, _ = problem("chain")
    r = L.newton_schulz_inv_sqrt(S, s.H.b, 0.0, 1e-14, 1)
    assert r.status == L.STATUS_NOT_CONVERGED and r.iters == 1


# ---------------------------------------------------------------- perturbed overlap (displacement)
def displaced(name="chain"):
    s, S, H, _ = problem(name)
    atom = s.H.nb // 2
    H1b, S1b = W.make_displacement(s, atom)
    return s, S, H, dense(H1b), dense(S1b)


def test_derivative_of_the_inverse_square_root():
    s, S, H, H1, S1 = displaced("cube")
    r = L.newton_schulz_response(S, [S1], s.H.b, 0.0, 1e-14, 50)
    assert r.status == L.STATUS_OK
    h = 1e-5
    fd = (inv_sqrt(S + h * S1) - inv_sqrt(S - h * S1)) / (2 * h)
    np.testing.assert_allclose(r.Z1[0], fd, atol=1e-8)
    # d(Z S Z) = 0
    Z, Z1 = r.Z, r.Z1[0]
    np.testing.assert_allclose(Z1 @ S @ Z + Z @ S1 @ Z + Z @ S @ Z1, 0.0, atol=1e-11)
    assert np.array_equal(Z1, Z1.T)


def test_orthogonal_perturbation_is_the_derivative_of_the_orthogonal_form():
    s, S, H, H1, S1 = displaced("chain")
    o = L.lowdin_response(S, [S1], H, [H1], s.H.b, 0.0, 1e-14, 50)
    h = 1e-5
    orth = lambda x: inv_sqrt(S + x * S1) @ (H + x * H1) @ inv_sqrt(S + x * S1)
    np.testing.assert_allclose(o.H1[0], (orth(h) - orth(-h)) / (2 * h), atol=1e-8)


def test_displacement_response_is_the_derivative_of_the_generalised_projector():
    # P1 = Z1 X0 Z + Z X1 Z + Z X0 Z1 with X0, X1 the orthogonal projector and
    # its response to H1_orth, against finite differences of the projector of
    # H C = S C E when both H and S move
    s, S, H, H1, S1 = displaced("chain")
    b = s.H.b
    o = L.lowdin_response(S, [S1], H, [H1], b, 0.0, 1e-14, 50)
    X0 = E.exact_projector(o.H, s.n_occ)
    X1 = E.exact_response(o.H, o.H1[0], s.n_occ)
    P1 = L.congruence_response(o.Z, o.Z1[0], X0, X1, b, 0.0)
    h = 1e-5
    fd = (generalised_projector(H + h * H1, S + h * S1, s.n_occ)
          - generalised_projector(H - h * H1, S - h * S1, s.n_occ)) / (2 * h)
    np.testing.assert_allclose(P1, fd, atol=1e-7)
    assert np.abs(P1).max() > 1e-3                   # the check has something to check


def test_unchanged_overlap_reduces_to_the_field_case():
    s, S, H, H1, _ = displaced("chain")
    z = np.zeros_like(S)
    o = L.lowdin_response(S, [z], H, [H1], s.H.b, 1e-8, 1e-12, 50)
    f = L.lowdin(S, H, [H1], s.H.b, 1e-8, 1e-12, 50)
    assert np.array_equal(o.Z1[0], z)
    np.testing.assert_allclose(o.H1[0], f.H1[0], atol=1e-14)
    assert np.array_equal(o.Z, f.Z) and o.iters == f.iters


# ---------------------------------------------------------------- the mirrored symmetric products
def _ns_products(S, b, eps, iters=12):
    """Newton-Schulz iterates (mirrored reading) and, for every product of
    the iteration, the plain computed product A @ B next to the mirrored one."""
    N = S.shape[0]
    lam = L.gershgorin_upper(S)
    Y, Z = S / lam, np.eye(N)
    pairs = []
    prev = None
    for _ in range(iters):
        M = L.symmetric_product(Z, Y, b, eps)
        pairs.append((Z @ Y, M))
        resid = np.linalg.norm(M - np.eye(N)) / np.sqrt(N)
        if resid < 1e-13 or (prev is not None and resid > 0.5 * prev):
            break
        prev = resid
        T = 0.5 * (3.0 * np.eye(N) - M)
        Yn, Zn = L.symmetric_product(Y, T, b, eps), L.symmetric_product(Z, T, b, eps)
        pairs += [(Y @ T, Yn), (Z @ T, Zn)]
        Y, Z = Yn, Zn
    return pairs


@pytest.mark.parametrize("name", ["chain", "cube"])
def test_mirrored_products_are_plain_products_at_eps_zero(name):
    # without the filter the products of the iteration are exact functions of
    # S, symmetric up to rounding: mirroring the upper blocks discards only that
    s, S, _, _ = problem(name)
    for C, Cm in _ns_products(S, s.H.b, 0.0):
        assert np.abs(C - C.T).max() < 1e-14
        assert np.abs(C - Cm).max() < 1e-14


@pytest.mark.parametrize("name", ["chain", "cube"])
@pytest.mark.parametrize("eps", [1e-8, 1e-6, 1e-4])
def test_mirror_discards_less_than_eps(name, eps):
    # with the filter: Z = f(S) + E_Z and Y = g(S) + E_Y, where f(S), g(S)
    # commute and E_Z, E_Y hold what the filter removed (blocks of norm < eps,
    # sparse in every block row).  Z Y - (Z Y)^T = [Z, Y] = [E_Z, g] + [f, E_Y]
    # + [E_Z, E_Y] then stays of the order of eps, and the mirror keeps the
    # upper half of the product: off the upper blocks it moves each element
    # by |C - C^T|.  Within the filter's own resolution (below eps) the
    # mirrored product is the plain product of the iteration.
    s, S, _, _ = problem(name)
    worst = 0.0
    for C, Cm in _ns_products(S, s.H.b, eps):
        Cf = L.product(C, np.eye(C.shape[0]), s.H.b, eps)   # plain product, filtered
        worst = max(worst, np.abs(C - C.T).max())
        # mirrored vs plain: differences only where the blocks differ by the
        # asymmetry, or where one reading dropped a block near eps
        assert np.abs(Cf - Cm).max() < eps
    assert worst < eps


@pytest.mark.parametrize("name", ["chain", "cube"])
@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_mirrored_inverse_square_root_is_the_plain_one_within_eps(name, eps):
    # the whole iteration, every product plain (no mirror, each block filtered
    # on its own) against the mirrored reading used by the library
    s, S, _, _ = problem(name)
    a = L.newton_schulz_inv_sqrt(S, s.H.b, eps, 1e-12, 40)
    p = L.newton_schulz_inv_sqrt(S, s.H.b, eps, 1e-12, 40, mirror=False)
    assert a.iters == p.iters and a.status == p.status
    assert np.abs(a.Z - p.Z).max() < eps
    assert np.abs(p.Z - p.Z.T).max() < eps        # the plain result is symmetric within eps
