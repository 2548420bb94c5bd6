"""Pins of the oracle's D+S functions (a binary64 leading part and a binary32
trailing part, the format of Section 4.4's GPU comparison) against exact
rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

import workload as W


def rn(x: Fraction, p: int, emin: int) -> Fraction:
    """x rounded to p significand bits (minimum exponent emin), ties to even."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    lsb = max(e - (p - 1), emin)
    q = a / Fraction(2) ** lsb
    f = q.numerator // q.denominator
    r = q - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return sign * f * Fraction(2) ** lsb


def test_ds_round_against_rationals(orc):
    """hi = RN53(v), lo = RN24(v - hi) of the exact sum, including sums whose
    second part is not representable in binary32 and halfway cases."""
    X = W.gen_matrix("qd", 40, 3, E=20, seed=5)  # 4-term expansions
    X[1, 0, 0] = 2.0 ** -53 * X[0, 0, 0] * 0.75  # an exact halfway-type second part
    X[2:, 0, 0] = 0.0
    hi, lo = orc.ds_round(X)
    for idx in np.ndindex(hi.shape):
        v = sum(Fraction(float(X[(r,) + idx])) for r in range(X.shape[0]))
        h = rn(v, 53, -1074)
        assert Fraction(float(hi[idx])) == h, idx
        assert Fraction(float(lo[idx])) == rn(v - h, 24, -149), idx
        assert abs(Fraction(float(lo[idx]))) <= abs(h) * Fraction(2) ** -53


def test_ds_generator_is_normalized():
    hi, lo = W.gen_ds(50, 7, E=16, seed=3)
    assert hi.dtype == np.float64 and lo.dtype == np.float32
    assert np.all(np.abs(lo.astype(np.float64)) <= np.abs(hi) * 2.0 ** -53)
    assert np.any(lo != 0)


@pytest.mark.parametrize("m,n,k", [(3, 4, 5), (7, 2, 33)])
def test_naive_ds_against_rationals(orc, m, n, k):
    """The D+S triple loop: C is the D+S rounding (hi = RN53, lo = RN24 of the
    rest) of a DD accumulation whose error is at most k 2^-103 (|A||B|): so
    |C - AB| <= (k 2^-103 + 2^-76) (|A||B|), and C's parts are the D+S
    rounding of some value within k 2^-103 (|A||B|) of AB."""
    Ahi, Alo = W.gen_ds(m, k, E=8, seed=11, operand="A")
    Bhi, Blo = W.gen_ds(k, n, E=8, seed=11, operand="B")
    Chi, Clo = orc.gemm_naive_ds(Ahi, Alo, Bhi, Blo)
    for i in range(m):
        for j in range(n):
            ab = sum((Fraction(float(Ahi[0, p, i])) + Fraction(float(Alo[0, p, i])))
                     * (Fraction(float(Bhi[0, j, p])) + Fraction(float(Blo[0, j, p]))) for p in range(k))
            absab = sum(abs(Fraction(float(Ahi[0, p, i])) + Fraction(float(Alo[0, p, i])))
                        * abs(Fraction(float(Bhi[0, j, p])) + Fraction(float(Blo[0, j, p]))) for p in range(k))
            c = Fraction(float(Chi[0, j, i])) + Fraction(float(Clo[0, j, i]))
            assert abs(c - ab) <= (k * Fraction(2) ** -103 + Fraction(2) ** -76) * absab, (i, j)
            assert abs(Fraction(float(Clo[0, j, i]))) <= abs(Fraction(float(Chi[0, j, i]))) * Fraction(2) ** -53


def test_naive_ds_rows_subset_and_exact_check(orc):
    """Selected rows equal the full result's rows, and the D+S result read as
    a DD pair passes the exact check within the same bound."""
    m, n, k = 9, 6, 50
    Ahi, Alo = W.gen_ds(m, k, E=16, seed=12, operand="A")
    Bhi, Blo = W.gen_ds(k, n, E=16, seed=12, operand="B")
    Chi, Clo = orc.gemm_naive_ds(Ahi, Alo, Bhi, Blo)
    rows = [8, 0, 3]
    Shi, Slo = orc.gemm_naive_ds(Ahi, Alo, Bhi, Blo, rows=rows)
    assert np.array_equal(Shi, Chi[:, :, rows]) and np.array_equal(Slo, Clo[:, :, rows])
    A, B, C = orc.ds_as_dd(Ahi, Alo), orc.ds_as_dd(Bhi, Blo), orc.ds_as_dd(Chi, Clo)
    diff, absab, _ = orc.exact_check(A, B, C)
    assert np.all(diff <= (k * 2.0 ** -103 + 2.0 ** -76) * absab)
    assert np.any(diff > 0)
