"""Pins of the oracle's exact LU checks (used by the LU tests of Section 4.6's
application): the backward error is zero for factors whose product is the
matrix exactly and equals the planted error otherwise; the exact solve
satisfies A x = b in rationals."""
from fractions import Fraction

import numpy as np

import oracle.exact as X


def _dd_matrix(M):
    """(2, n, n) planes (column-major) holding the double matrix M[i][j]."""
    n = len(M)
    A = np.zeros((2, n, n))
    for i in range(n):
        for j in range(n):
            A[0, j, i] = M[i][j]
    return A


def test_backward_error_exact_and_planted():
    rng = np.random.default_rng(3)
    n = 6
    # dyadic unit-lower L and upper U with small entries: L U is exact in binary64
    L = np.tril(rng.integers(-4, 5, size=(n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(1, 9, size=(n, n)) / 4.0)
    A = L @ U
    LU = np.tril(L, -1) + U
    assert X.lu_backward_error(_dd_matrix(A.tolist()), _dd_matrix(LU.tolist())) == 0.0
    # plant an error of 2^-60 in U[2][4] through the lo plane of the factors
    LUd = _dd_matrix(LU.tolist())
    LUd[1, 4, 2] = 2.0 ** -60
    got = X.lu_backward_error(_dd_matrix(A.tolist()), LUd)
    # |A - L U|_{i,4} = |L_{i,2}| 2^-60 for i >= 2; |L||U| is exact
    want = max(Fraction(abs(L[i][2])) * Fraction(2) ** -60 /
               sum(Fraction(abs(L[i][q] * (U[q][4] + (2.0 ** -60 if q == 2 else 0)))) for q in range(min(i, 4) + 1))
               for i in range(2, n))
    assert got == float(want)


def test_backward_error_sampled_entries():
    """The sampled form agrees with the full one: zero off the planted column,
    the planted ratio on it, and every entry listed gives the full result."""
    rng = np.random.default_rng(4)
    n = 7
    L = np.tril(rng.integers(-4, 5, size=(n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(rng.integers(1, 9, size=(n, n)) / 4.0)
    A = _dd_matrix((L @ U).tolist())
    LUd = _dd_matrix((np.tril(L, -1) + U).tolist())
    LUd[1, 5, 3] = 2.0 ** -70  # U[3][5] + 2^-70: entries (i, 5) with i >= 3 change
    full = X.lu_backward_error(A, LUd)
    assert full > 0
    every = [(i, j) for i in range(n) for j in range(n)]
    assert X.lu_backward_error(A, LUd, entries=every) == full
    assert X.lu_backward_error(A, LUd, entries=[(i, j) for i, j in every if j != 5]) == 0.0
    col = [(i, 5) for i in range(n)]
    assert X.lu_backward_error(A, LUd, entries=col) == full
    assert X.lu_backward_error(A, LUd, entries=[(0, 5), (1, 5), (2, 5)]) == 0.0


def test_solve_exact_satisfies_system():
    rng = np.random.default_rng(5)
    n = 7
    M = (rng.random((n, n)) + n * np.eye(n)).tolist()
    A = _dd_matrix(M)
    b = np.zeros((2, n))
    b[0] = rng.random(n)
    b[1] = b[0] * 2.0 ** -60
    x = X.solve_exact(A, b)
    for i in range(n):
        lhs = sum((Fraction(M[i][j]) * x[j] for j in range(n)), Fraction(0))
        assert lhs == Fraction(float(b[0, i])) + Fraction(float(b[1, i]))
