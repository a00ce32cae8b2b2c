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
