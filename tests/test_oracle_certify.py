"""Pins of the a-posteriori error bound's truncation part (the oracle's
``certificate_terms``): with D slices per row and column (Algorithm 1 and the
pairs a + b <= D + 1 of Section 3), the exact |C_tri - AB| never exceeds
T1 + T2 + T3 (left-out pairs, and remainders), checked in exact rational
arithmetic; and inputs are built on which dropping either part would fail."""
from fractions import Fraction

import numpy as np
import pytest

import workload as W


def _entries(m, n):
    return [(i, j) for i in range(m) for j in range(n)]


@pytest.mark.parametrize("fmt,E,D", [("dd", 16, 2), ("dd", 16, 3), ("dd", 0, 2), ("td", 8, 2), ("qd", 16, 3),
                                     ("ts", 16, 3), ("ts", 8, 5)])
def test_truncation_within_bound(orc, fmt, E, D):
    m, n, k = 5, 4, 13
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=m + n + k + D)
    tr, t1, t23, _ = orc.certificate_terms(A, B, D)
    ratios = []
    for i, j in _entries(m, n):
        bound = t1[i][j] + t23[i][j]
        assert tr[i][j] <= bound, (i, j)
        if bound > 0:
            ratios.append(tr[i][j] / bound)
    # the bound is an estimate, not a formality: within 2^8 of the truth somewhere
    assert max(ratios) > Fraction(1, 256)


@pytest.mark.parametrize("fmt,E,D", [("dd", 16, 6), ("dd", 16, 9), ("td", 0, 10), ("qd", 8, 12)])
def test_truncation_within_bound_int8(orc, fmt, E, D):
    """The same bound with INT8 digit planes as slices (grid 2^(E - 6 - 7 (s - 1)))."""
    m, n, k = 5, 4, 13
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=7 + D)
    tr, t1, t23, _ = orc.certificate_terms(A, B, D, form="int8")
    for i, j in _entries(m, n):
        assert tr[i][j] <= t1[i][j] + t23[i][j], (i, j)
    # one digit: nothing is left out, the remainder bound alone carries it
    tr1, t11, t231, _ = orc.certificate_terms(A, B, 1, form="int8")
    assert all(t11[i][j] == 0 and tr1[i][j] <= t231[i][j] for i, j in _entries(m, n))
    assert any(tr1[i][j] > 0 for i, j in _entries(m, n))


def test_remainder_terms_bound_d1(orc):
    """D = 1 leaves out no pair (T1 = 0): the truncation is the remainders'
    alone, and T2 + T3 by itself must bound it."""
    m, n, k = 4, 3, 9
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=3)
    tr, t1, t23, _ = orc.certificate_terms(A, B, 1)
    assert all(t1[i][j] == 0 for i, j in _entries(m, n))
    assert any(tr[i][j] > 0 for i, j in _entries(m, n))
    assert all(tr[i][j] <= t23[i][j] for i, j in _entries(m, n))


def test_left_out_pairs_bounded_by_t1(orc):
    """Elements that two slices hold exactly (D = 2): the remainders are exactly
    zero, so the truncation is the left-out pair (2, 2) alone, and T1 by itself
    must bound it (a wrong pair set or exponent in T1 fails here)."""
    m, n, k = 3, 3, 5
    S = 53
    b = S - orc.rho(S, k)  # bits per slice
    rng = np.random.default_rng(1)
    A = np.zeros((2, k, m))
    B = np.zeros((2, n, k))
    # 1 + (small integer) 2^-(b + 3): the second slice holds the tail exactly
    A[0] = 1.0 + rng.integers(1, 8, size=(k, m)) * 2.0 ** -(b + 3)
    B[0] = 1.0 + rng.integers(1, 8, size=(n, k)) * 2.0 ** -(b + 3)
    _, _, ra = orc.split_plain(A, 2, "rows", want_resid=True)
    _, _, rb = orc.split_plain(B, 2, "cols", want_resid=True)
    assert not ra.any() and not rb.any()
    tr, t1, _, _ = orc.certificate_terms(A, B, 2)
    assert all(0 < tr[i][j] <= t1[i][j] for i, j in _entries(m, n))
    # and within a factor 2^6 of it (all second slices share one sign)
    assert all(tr[i][j] * 64 >= t1[i][j] for i, j in _entries(m, n))


@pytest.mark.parametrize("fmt,E,D", [("dd", 16, 4), ("qd", 8, 5), ("ts", 16, 5)])
def test_truncation_within_bound_any_staircase(orc, fmt, E, D):
    """Pair sets other than the triangle (the per-tile sets chosen from the
    data): for random staircases per entry, from the empty set to the full
    D x D square, the exact |C_P - AB| stays within T1 (over every pair left
    out) + T2 + T3; the full square leaves only the remainder terms, the empty
    set only |AB| itself."""
    m, n, k = 4, 3, 11
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=31 + D)
    rng = np.random.default_rng(D)
    sets = {}
    for i, j in _entries(m, n):
        counts = np.sort(rng.integers(0, D + 1, D))[::-1]  # non-increasing: a staircase
        sets[(i, j)] = [int(c) for c in counts]
    sets[(0, 0)] = [D] * D
    sets[(m - 1, n - 1)] = [0] * D
    tr, t1, t23, absab = orc.certificate_terms(A, B, D, pairs=lambda i, j: sets[(i, j)])
    for i, j in _entries(m, n):
        assert tr[i][j] <= t1[i][j] + t23[i][j], (i, j, sets[(i, j)])
    assert t1[0][0] == 0
    import oracle.exact as X
    Av, Bv = X.matrix_values(A), X.matrix_values(B)
    ab = sum((Av[m - 1][p] * Bv[p][n - 1] for p in range(k)), Fraction(0))
    assert tr[m - 1][n - 1] == abs(ab)
    # the triangle given explicitly is the default
    tri = orc.certificate_terms(A, B, D, pairs=lambda i, j: [D - a for a in range(D)])
    assert tri == orc.certificate_terms(A, B, D)
