"""The block-sparse products behind the Loewdin entry points on random
patterns: tc2_congruence (Z X Z) and tc2_congruence_response (Z1 X Z +
Z X1 Z + Z X Z1) against the oracle's dense products with the same filter,
for block sizes 1 to 16, empty rows and columns, and several thresholds."""
import numpy as np
import pytest

from oracle import lowdin as L
from oracle import tc2_oracle as O
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def random_symmetric(rng, nb, b, density, diag=True):
    """A random symmetric BSR matrix: each upper pair (I, J) present with the
    given probability, blocks of random values (transposed below)."""
    mask = np.triu(rng.random((nb, nb)) < density, k=1)
    blocks = {}
    for I, J in zip(*np.nonzero(mask)):
        v = rng.standard_normal((b, b)) * rng.choice([1.0, 1e-2, 1e-4])
        blocks[(I, J)] = v
        blocks[(J, I)] = v.T
    if diag:
        for I in range(nb):
            g = rng.standard_normal((b, b))
            blocks[(I, I)] = 0.5 * (g + g.T) + 2.0 * np.eye(b)
    rp, ci, va = [0], [], []
    for I in range(nb):
        for J in sorted(j for (i, j) in blocks if i == I):
            ci.append(J)
            va.append(blocks[(I, J)])
        rp.append(len(ci))
    return W.BSR(nb, b, np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int32),
                 np.array(va, dtype=np.float64).reshape(-1, b, b))


def dense(m):
    return O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val)


def pattern(X, b):
    nb = X.shape[0] // b
    return np.abs(X.reshape(nb, b, nb, b)).sum(axis=(1, 3)) > 0


CASES = [(seed, nb, b, density, eps)
         for seed, (nb, b, density, eps) in enumerate([
             (1, 1, 1.0, 0.0), (7, 1, 0.3, 0.0), (23, 3, 0.2, 1e-3), (17, 8, 0.15, 1e-6),
             (12, 13, 0.3, 1e-2), (9, 16, 0.4, 0.0), (40, 5, 0.05, 1e-4), (33, 2, 0.5, 1e-1)])]


@pytest.mark.parametrize("seed,nb,b,density,eps", CASES)
def test_congruence_on_random_patterns(seed, nb, b, density, eps):
    rng = np.random.default_rng(seed)
    Z = random_symmetric(rng, nb, b, density)
    X = random_symmetric(rng, nb, b, density, diag=rng.random() < 0.5)
    got = dense(T.congruence(Z, X, eps=eps))
    want = L.congruence(dense(Z), dense(X), b, eps)
    assert np.array_equal(got, got.T)
    assert np.array_equal(pattern(got, b), pattern(want, b))
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("seed,nb,b,density,eps", CASES[2:6])
def test_congruence_response_on_random_patterns(seed, nb, b, density, eps):
    rng = np.random.default_rng(100 + seed)
    Z = random_symmetric(rng, nb, b, density)
    Z1 = random_symmetric(rng, nb, b, density, diag=False)
    X = random_symmetric(rng, nb, b, density)
    X1 = random_symmetric(rng, nb, b, density, diag=False)
    got = dense(T.congruence_response(Z, Z1, X, X1, eps=eps))
    want = L.congruence_response(dense(Z), dense(Z1), dense(X), dense(X1), b, eps)
    assert np.array_equal(got, got.T)
    assert np.array_equal(pattern(got, b), pattern(want, b))
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
