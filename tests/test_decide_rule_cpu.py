"""The stopping rule that the device-side decision kernel applies
(paper_2009_03551_amd/csrc/tc2_decide_rule.h), built with gcc through a small
shim, against the oracle's stopping rule (``tc2_oracle.stopping_rule`` plus
the iteration limit) on hand-scripted and random histories of the band
energies, the response traces and iota.  The two are separate
implementations of the same readings of Sec. 2.3 (tolerance test, then stall
guard), so a change of order, of an index (k - 1 for k - 2) or of a
comparison's strictness in either shows here."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import tc2_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM = os.path.join(ROOT, "tests", "c", "decide_rule_shim.c")
ENAN, NOT_CONVERGED = -6, 1


@pytest.fixture(scope="module")
def rule(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("rule") / "libdecide_rule.so")
    r = subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-shared",
                        "-fPIC", "-o", so, SHIM, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    lib = C.CDLL(so)
    f = lib.decide_replay
    f.restype = C.c_int
    f.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                  C.POINTER(C.c_int), C.c_double, C.c_int, C.POINTER(C.c_int)]

    def run(D, e, iota, tol, max_iter, bad=None):
        e = np.ascontiguousarray(e, dtype=np.float64)
        iota = np.ascontiguousarray(iota, dtype=np.float64)
        st = C.c_int(0)
        bp = None
        if bad is not None:
            b = np.ascontiguousarray(bad, dtype=np.int32)
            bp = b.ctypes.data_as(C.POINTER(C.c_int))
        k = f(D, len(iota), e.ctypes.data_as(C.POINTER(C.c_double)),
              iota.ctypes.data_as(C.POINTER(C.c_double)), bp, tol, max_iter, C.byref(st))
        return (k, st.value) if k > 0 else (0, None)
    return run


def oracle(D, e, iota, tol, max_iter):
    """The oracle's decision: its stopping rule after each update, then the
    iteration limit."""
    def split(row):
        return (row[0], list(row[1:1 + D]), list(row[1 + D:1 + 2 * D]))
    for k in range(1, len(iota) + 1):
        st = O.stopping_rule(k, split(e[k - 1]), split(e[k]), list(iota[:k]), tol)
        if st is not None:
            return k, st
        if k >= max_iter:
            return k, NOT_CONVERGED
    return 0, None


def rows(D, seq):
    """History rows from (E0, [E1], [alpha]) tuples."""
    return np.array([[a] + list(b) + list(c) for a, b, c in seq], dtype=np.float64).reshape(
        len(seq), 1 + 2 * D)


def test_hand_cases(rule):
    tol = 1e-9
    big = [0.9, 0.8, 0.7, 0.6, 0.5, 0.4]
    # converges at the second update, not at the first
    e = rows(1, [(-1.0, [0.3], [-2.0]), (-1.0, [0.3], [-2.0]), (-1.0, [0.3], [-2.0])])
    assert rule(1, e, [0.5, 0.4], tol, 50) == (2, 0)
    # strict: a change of exactly tol does not stop
    e = rows(0, [(0.0, [], []), (0.0, [], []), (tol, [], []), (tol, [], [])])
    assert rule(0, e, [0.9, 0.8, 0.7], tol, 50) == (3, 0)
    # a change of alpha alone (update 2), or of Tr(X1 H) alone (update 3),
    # blocks convergence; update 4 changes nothing and stops
    e = rows(1, [(-1.0, [0.3], [-2.0])] * 2 + [(-1.0, [0.3], [-2.0 + 1e-6])] +
             [(-1.0, [0.3 + 1e-6], [-2.0 + 1e-6])] * 2)
    assert rule(1, e, big[:4], tol, 50) == (4, 0)
    assert oracle(1, e, big[:4], tol, 50) == (4, 0)
    # the stall guard fires on |iota_3| >= |iota_1| and not on the reverse
    grow = rows(0, [(float(i), [], []) for i in range(5)])
    assert rule(0, grow, [0.3, 0.6, 0.4], tol, 50) == (3, 2)
    assert rule(0, grow, [0.5, 0.3, 0.4], tol, 50) == (0, None)
    # no guard at |iota| >= 1, and the tolerance test comes first
    assert rule(0, grow, [1.5, 1.2, 1.5], tol, 50) == (0, None)
    flat = rows(0, [(1.0, [], [])] * 4)
    assert rule(0, flat, [0.3, 0.6, 0.4], tol, 50) == (2, 0)
    # the iteration limit, and a non-finite product value
    assert rule(0, grow, big[:4], tol, 3) == (3, NOT_CONVERGED)
    assert rule(0, grow, big[:4], tol, 50, bad=[0, 1, 0, 0]) == (2, ENAN)
    # every hand case agrees with the oracle where the oracle has the notion
    for D, e, io, mi in ((0, grow, [0.3, 0.6, 0.4], 50), (0, grow, [0.5, 0.3, 0.4], 50),
                         (0, flat, [0.3, 0.6, 0.4], 50), (0, grow, big[:4], 3)):
        assert rule(D, e, io, tol, mi) == oracle(D, e, io, tol, mi)


@pytest.mark.parametrize("D", [0, 1, 3])
def test_random_histories(rule, D):
    rng = np.random.default_rng(17 + D)
    stops = {0: 0, 1: 0, 2: 0, None: 0}
    for case in range(600):
        n = int(rng.integers(1, 31))
        tol = 10.0 ** rng.uniform(-10, -4)
        # values approach a limit with steps that shrink around tol, some
        # of them exactly tol or zero; iota shrinks with noise and exact ties
        steps = tol * 10.0 ** rng.uniform(-3, 4, size=(n, 1 + 2 * D))
        steps[rng.random(size=steps.shape) < 0.05] = tol
        steps[rng.random(size=steps.shape) < 0.05] = 0.0
        sign = rng.choice([-1.0, 1.0], size=steps.shape)
        e = np.vstack([rng.normal(size=(1, 1 + 2 * D)),
                       np.zeros((n, 1 + 2 * D))])
        for u in range(n):
            e[u + 1] = e[u] + sign[u] * steps[u]
        iota = np.abs(rng.normal(size=n)) * 10.0 ** rng.uniform(-3, 1, size=n)
        ties = rng.random(size=n) < 0.2
        for u in range(2, n):
            if ties[u]:
                iota[u] = iota[u - 2] * rng.choice([-1.0, 1.0])
        max_iter = int(rng.integers(1, 40))
        got = rule(D, e, iota, tol, max_iter)
        want = oracle(D, e, iota, tol, max_iter)
        assert got == want, (case, n, tol, max_iter, got, want)
        stops[got[1]] += 1
    # the histories reach every outcome
    assert all(v > 0 for v in stops.values()), stops
