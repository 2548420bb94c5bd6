"""Exact pure-Python references that pin the C oracle (test infrastructure).

Everything here is exact rational or integer arithmetic (``fractions`` and
Python ``int``), or plain IEEE arithmetic on Python floats / numpy float32
where the method itself prescribes a floating-point step.  It is written
independently of ``oracle.c`` so the two can be compared; it is slow and meant
for small inputs only.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def value(comps) -> Fraction:
    """Exact value of an expansion (a sequence of binary64/binary32 components)."""
    return sum((Fraction(float(x)) for x in comps), Fraction(0))


def matrix_values(X) -> list:
    """Exact element values of a ``(c, cols, rows)`` array: ``V[i][p]``."""
    c, cols, rows = X.shape
    return [[value(X[:, p, i]) for p in range(cols)] for i in range(rows)]


def matmul_fraction(A, B):
    """Exact ``A B`` for ``(c, k, m)`` and ``(c, n, k)`` inputs, as ``C[i][j]`` Fractions."""
    Av = matrix_values(A)
    Bv = matrix_values(B)  # Bv[p][j]
    m, k = len(Av), len(Av[0]) if Av else 0
    n = B.shape[1]
    return [[sum((Av[i][p] * Bv[p][j] for p in range(k)), Fraction(0)) for j in range(n)] for i in range(m)]


def _scaled_ints(X):
    """Every element of X as an integer times 2**q for one common q."""
    comps = X.astype(np.float64)
    q = None
    nz = comps[comps != 0]
    for v in nz.ravel():
        m, e = math.frexp(float(v))
        qq = e - 53
        q = qq if q is None else min(q, qq)
    if q is None:
        q = 0
    c, cols, rows = X.shape
    ints = [[0] * cols for _ in range(rows)]
    for i in range(rows):
        for p in range(cols):
            s = 0
            for r in range(c):
                v = float(comps[r, p, i])
                if v != 0:
                    s += int(Fraction(v) * (Fraction(2) ** -q))
            ints[i][p] = s
    return ints, q


def matmul_exact_int(A, B):
    """Exact ``A B`` by scaled Python integers: returns ``(Cint, q)`` with
    ``C[i][j] = Cint[i][j] * 2**q`` (fast enough for 128^3)."""
    Ai, qa = _scaled_ints(A)  # Ai[i][p]
    Bi, qb = _scaled_ints(B)  # Bi[p][j] (rows of B are p)
    m = len(Ai)
    k = len(Ai[0]) if m else 0
    n = B.shape[1]
    Bt = [[Bi[p][j] for p in range(k)] for j in range(n)]
    C = [[sum(x * y for x, y in zip(Ai[i], Bt[j])) for j in range(n)] for i in range(m)]
    return C, qa + qb


def rho_exact(S: int, k: int) -> int:
    """Smallest integer r with r >= (S + log2 k)/2, i.e. 2**(2r - S) >= k (no floating point)."""
    r = 0
    while True:
        if 2 * r - S >= 0 and (1 << (2 * r - S)) >= k:
            return r
        if 2 * r - S < 0 and k <= 0:
            return r
        r += 1


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def renorm_py(x, f32: bool = False):
    """The same written renormalization as the oracle: a bottom-up TwoSum pass,
    then a top-down TwoSum pass that emits a term whenever its error is nonzero."""
    t = np.float32 if f32 else float
    x = [t(v) for v in x]
    n = len(x)
    e = [t(0)] * n
    s = x[-1]
    for i in range(n - 2, -1, -1):
        s, e[i + 1] = _two_sum(x[i], s)
    out = []
    cur = s
    for i in range(1, n):
        cur, err = _two_sum(cur, e[i])
        if err != 0:
            out.append(cur)
            cur = err
    out.append(cur)
    out += [t(0)] * (n - len(out))
    return out


def split_vector_py(vec, D: int, f32: bool = False, last_remainder: bool = False):
    """Algorithm 1's split of one row/column (a list of component tuples).

    Returns ``(slices[D][len], exps[D], residual[len][c])`` with the same
    readings as the C oracle (D passes, remainder dropped, mu = 0 gives a zero
    slice and exponent None).  ``last_remainder``: the D-th slice is instead the
    leading component of the residual after D - 1 passes (Algorithm 1 as
    printed).
    """
    t = np.float32 if f32 else float
    S = 24 if f32 else 53
    ln = len(vec)
    r = rho_exact(S, ln)
    R = [[t(v) for v in comps] for comps in vec]
    slices, exps = [], []
    for a in range(D):
        mu = max((abs(x[0]) for x in R), default=t(0))
        if mu == 0:
            slices.append([t(0)] * ln)
            exps.append(None)
            continue
        fr = Fraction(float(mu))
        e = 0
        while Fraction(2) ** e < fr:
            e += 1
        while Fraction(2) ** (e - 1) >= fr:
            e -= 1
        exps.append(e)
        tau = t(2.0 ** (e + r))
        row = []
        for x in R:
            lead = x[0]
            sl = lead if (last_remainder and a == D - 1) else (lead + tau) - tau
            row.append(sl)
            x[0] = lead - sl
            x[:] = renorm_py(x, f32)
        slices.append(row)
    return slices, exps, R


def rne(q: Fraction) -> int:
    """Nearest integer to the rational q, ties to even."""
    fl = math.floor(q)
    frac = q - fl
    return fl + 1 if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2 == 1) else fl


def int8_digits_py(comps_list, D: int):
    """INT8 digits of one row/column with exact rationals: ``(digits[len][D], E)``.

    Same written rule as the oracle: E = 1 + max ilogb of the leading
    components; digit s is the exact residual (the whole expansion at s = 1)
    divided by u_s = 2^(E - 6 - 7 (s - 1)) and rounded to nearest (ties to
    even), and the residual loses d_s u_s.
    """
    lead = [float(c[0]) for c in comps_list]
    nz = [x for x in lead if x != 0]
    if not nz:
        return [[0] * D for _ in comps_list], None
    E = max(math.frexp(x)[1] for x in nz)  # frexp exponent = ilogb + 1
    out = []
    for comps in comps_list:
        R = sum((Fraction(float(v)) for v in comps), Fraction(0))
        digs = []
        for s in range(1, D + 1):
            u = Fraction(2) ** (E - 6 - 7 * (s - 1))
            d = rne(R / u)
            digs.append(d)
            R -= d * u
        out.append(digs)
    return out, E


def lu_backward_error(A, LU, entries=None) -> float:
    """Largest |A - L U|_ij / (|L||U|)_ij over the entries, exactly: A and LU
    are ``(c, n, n)`` expansions (component planes, column-major), LU holding
    the unit lower L below its diagonal and U on and above it (the blocked LU
    of Section 4.6).  ``entries``: the (i, j) pairs to check, else every entry
    (small n only)."""
    n = A.shape[2]
    if entries is None:
        entries = [(i, j) for i in range(n) for j in range(n)]

    def l_of(i, q):
        return Fraction(1) if i == q else value(LU[:, q, i])

    worst = Fraction(0)
    for i, j in entries:
        s, a = Fraction(0), Fraction(0)
        for q in range(min(i, j) + 1):
            t = l_of(i, q) * value(LU[:, j, q])  # L[i][q] U[q][j], q <= min(i, j)
            s += t
            a += abs(t)
        d = abs(value(A[:, j, i]) - s)
        if a > 0:
            worst = max(worst, d / a)
        elif d > 0:
            return math.inf
    return float(worst)


def solve_exact(A, b) -> list:
    """Exact solution of A x = b (Gaussian elimination in rationals, no
    pivoting needed for the nonsingular test matrices used); A ``(c, n, n)``,
    b ``(c, n)``.  Returns a list of Fractions."""
    n = A.shape[2]
    M = [row[:] for row in matrix_values(A)]
    y = [value(b[:, i]) for i in range(n)]
    for j in range(n):
        p = next(i for i in range(j, n) if M[i][j] != 0)
        if p != j:
            M[j], M[p] = M[p], M[j]
            y[j], y[p] = y[p], y[j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            if f:
                for q in range(j, n):
                    M[i][q] -= f * M[j][q]
                y[i] -= f * y[j]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - sum((M[i][q] * x[q] for q in range(i + 1, n)), Fraction(0))) / M[i][i]
    return x
