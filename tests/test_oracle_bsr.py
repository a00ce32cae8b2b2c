"""The block-list oracle against the dense oracle (two implementations of the
same updates of Eq. TC2 / TC2-CPSCF written independently: block sums over
common columns with mirrored upper blocks against dense products with the
dense filter) on systems small enough for both."""
import numpy as np
import pytest

from oracle import bsr_oracle as B
from oracle import tc2_oracle as O
from paper_2009_03551_amd import workloads as W


def dense(m):
    return O.bsr_to_dense(m.nb, m.b, m.row_ptr, m.col, m.val)


CASES = [
    ("chain64", dict(n=24), 1e-7),            # b = 8, one direction, long-range couplings
    ("cube10", dict(L=5, n_dir=3), 1e-6),     # b = 13, three directions
    ("cube10", dict(L=4, n_dir=2), 1e-5),     # coarser filter, two directions
]


@pytest.mark.parametrize("name,kw,eps", CASES)
def test_leading_updates_match_the_dense_oracle(name, kw, eps):
    s = W.config_system(name, eps=eps, **kw)
    b, nb, D = s.H.b, s.H.nb, len(s.H1)
    rows = sorted({0, nb // 3, nb // 2, nb - 1})
    lead = B.leading_updates(s.H, s.H1, s.n_occ, eps, rows, n_updates=3)
    H, H1s = dense(s.H), [dense(h) for h in s.H1]
    assert (lead.emin, lead.emax) == pytest.approx(O.gershgorin(H), abs=1e-13)
    for k in (1, 2, 3):
        o = O.tc2_solve(H, H1s, s.n_occ, b, eps, s.tol, replay=lead.branches[:k])
        assert o.branches == lead.branches[:k]
        # the oracle's own trace rule took these branches
        X0d = O.tc2_solve(H, H1s, s.n_occ, b, eps, s.tol, replay=lead.branches[:k - 1]).X0 \
            if k > 1 else O.tc2_init(H, H1s, *O.gershgorin(H))[0]
        assert (np.trace(X0d) >= s.n_occ) == (lead.branches[k - 1] == "S")
        assert lead.traces[k - 1] == pytest.approx(np.trace(X0d), rel=1e-13)
        mats = [o.X0] + list(o.X1)
        for I in rows:
            cols, vals = lead.rows[k - 1][I]
            # every block of the dense row: present in the block row, or zero
            for J in range(nb):
                p = np.searchsorted(cols, J)
                have = p < len(cols) and cols[p] == J
                for m in range(1 + D):
                    want = mats[m][I * b:(I + 1) * b, J * b:(J + 1) * b]
                    got = vals[p][m] if have else np.zeros((b, b))
                    np.testing.assert_allclose(got, want, atol=1e-12, rtol=0)
            # and the pattern holds no block that every matrix dropped
            for p, J in enumerate(cols):
                if J != I:
                    assert np.any(vals[p] != 0.0)
    # scalars of the first iterate, from the complete block rows
    o1 = O.tc2_solve(H, H1s, s.n_occ, b, eps, s.tol, replay=lead.branches[:1])
    E0, E1, al = O.band_energies(o1.X0, o1.X1, H, H1s)
    sc = lead.scalars1
    assert sc["tr_x0"] == pytest.approx(np.trace(o1.X0), rel=1e-13)
    assert sc["e0"] == pytest.approx(E0, rel=1e-12)
    np.testing.assert_allclose(sc["e1"], E1, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(sc["alpha"], al, rtol=1e-12)
    np.testing.assert_allclose(sc["tr_x1"], [np.trace(x) for x in o1.X1], atol=1e-12)


def test_upper_block_by_hand():
    # two 1x1 "blocks" per row: X = [[a, c], [c, d]] with one direction
    # X1 = [[p, q], [q, r]]:  (X X)_01 = a c + c d,  (X X1 + X1 X)_01 = a q + c r + p c + q d
    a, c, d, p, q, r = 0.7, -0.2, 0.4, 0.3, 0.5, -0.1
    X = {0: (np.array([0, 1]), np.array([[[[a]], [[p]]], [[[c]], [[q]]]])),
         1: (np.array([0, 1]), np.array([[[[c]], [[q]]], [[[d]], [[r]]]]))}
    C = B.upper_block(X, 0, 1)
    assert C[0, 0, 0] == pytest.approx(a * c + c * d)
    assert C[1, 0, 0] == pytest.approx(a * q + c * r + p * c + q * d)


def test_filter_keeps_diagonal_and_drops_per_matrix():
    C = np.zeros((2, 2, 2))
    C[0] = [[1e-3, 0.0], [0.0, 0.0]]          # X0 block above eps: kept
    C[1] = [[1e-7, 0.0], [0.0, 0.0]]          # X1 block below eps: dropped on its own
    Y = B.combine_and_filter(C, None, True, 1e-6, diag=False)
    assert Y[0, 0, 0] == 1e-3 and not Y[1].any()
    Yd = B.combine_and_filter(C, None, True, 1e-6, diag=True)
    assert Yd[1, 0, 0] == 1e-7
    # DOUBLE: 2 X - C with the old block
    old = np.ones((2, 2, 2))
    Z = B.combine_and_filter(C, old, False, 0.0, diag=False)
    np.testing.assert_allclose(Z, 2.0 * old - C)


def test_ball_on_a_chain():
    s = W.config_system("chain64", n=20)            # couplings up to 4 sites
    g = B.coupling_graph(s.H)
    assert list(B.ball(g, [10], 1)) == list(range(6, 15))
    assert list(B.ball(g, [0], 2)) == list(range(0, 9))
