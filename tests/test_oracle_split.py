"""Pins of the oracle's split (Section 3, Algorithm 1) against closed forms,
invariants, exact arithmetic and an independent Python implementation."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle.exact as X
import workload as W

FMTS = ["dd", "td", "qd", "ts"]


def test_rho_closed_form(orc):
    """ceil((S + log2 l)/2): the integer formula against an exact integer search, all l < 70000."""
    for S in (24, 53):
        r = 0
        for k in range(1, 70000):
            # smallest r with 2r >= S + log2 k  <=>  2^(2r - S) >= k
            while not (2 * r - S >= 0 and (1 << (2 * r - S)) >= k):
                r += 1
            assert orc.rho(S, k) == r, (S, k)
    assert [orc.rho(53, k) for k in (64, 1024, 4096)] == [30, 32, 33]
    assert orc.rho(24, 4096) == 18


def test_rho_gives_exact_products(orc):
    """k * 2^(2b) <= 2^S with b = S - rho: every slice-product sum fits the S-bit significand."""
    for S in (24, 53):
        for k in list(range(1, 300)) + [1000, 4096, 4097, 65535, 65536, 65537]:
            b = S - orc.rho(S, k)
            assert k * 2 ** (2 * b) <= 2 ** S


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("E", [0, 16])
def test_split_matches_independent_python(orc, fmt, E):
    m, k, D = 6, 11, 5
    A = W.gen_matrix(fmt, m, k, E=E, seed=5 + E, operand="A")
    sl, ex = orc.split_plain(A, D, "rows")
    f32 = fmt == "ts"
    for i in range(m):
        vec = [tuple(A[:, p, i]) for p in range(k)]
        s2, e2, _ = X.split_vector_py(vec, D, f32)
        for a in range(D):
            assert [float(v) for v in sl[a, :, i]] == [float(v) for v in s2[a]]
            assert ex[a, i] == (e2[a] if e2[a] is not None else orc.ZERO_EXP)
    B = W.gen_matrix(fmt, k, 4, E=E, seed=9, operand="B")
    slb, exb = orc.split_plain(B, D, "cols")
    for j in range(4):
        vec = [tuple(B[:, j, p]) for p in range(k)]
        s2, e2, _ = X.split_vector_py(vec, D, f32)
        for a in range(D):
            assert [float(v) for v in slb[a, j, :]] == [float(v) for v in s2[a]]


@pytest.mark.parametrize("fmt", FMTS)
def test_split_invariants(orc, fmt):
    """I1: slices plus remainder equal the input exactly.  I2: slice a lies on the
    grid 2^(e_a + rho - S) with |x| <= 2^e_a.  I3: the remainder after pass a is at
    most 2^(e_a + rho - S) (1 + 2^(1 - rho)).  e_1 = ceil(log2 max|x_0|)."""
    m, k, D = 7, 37, 6
    A = W.gen_matrix(fmt, m, k, E=16, seed=21, operand="A")
    f32 = fmt == "ts"
    S = 24 if f32 else 53
    rho = orc.rho(S, k)
    for Dp in range(1, D + 1):
        sl, ex, res = orc.split_plain(A, Dp, "rows", want_resid=True)
        for i in range(m):
            mu = max(abs(Fraction(float(A[0, p, i]))) for p in range(k))
            e_check = 0
            while Fraction(2) ** e_check < mu:
                e_check += 1
            while Fraction(2) ** (e_check - 1) >= mu:
                e_check -= 1
            assert ex[0, i] == e_check
            for p in range(k):
                x = X.value(A[:, p, i])
                tot = sum((Fraction(float(sl[a, p, i])) for a in range(Dp)), Fraction(0)) + X.value(res[:, p, i])
                assert tot == x  # I1
                for a in range(Dp):
                    e = int(ex[a, i])
                    q = Fraction(float(sl[a, p, i])) / Fraction(2) ** (e + rho - S)
                    assert q.denominator == 1 and abs(q) <= 2 ** (S - rho)  # I2
                eD = int(ex[Dp - 1, i])
                assert abs(X.value(res[:, p, i])) <= Fraction(2) ** (eD + rho - S) * (1 + Fraction(2) ** (1 - rho))  # I3


@pytest.mark.parametrize("fmt", ["dd", "ts"])
def test_first_slice_is_round_to_grid(orc, fmt):
    """(x + tau) - tau rounds x to nearest on the grid of fl(x + tau): step
    2^(e + rho - S + 1) for x >= 0 and 2^(e + rho - S) for x < 0, ties to an even
    multiple of the step (Algorithm 1's extraction, checked with rationals)."""
    m, k = 5, 64
    A = W.gen_matrix(fmt, m, k, E=8, seed=2, operand="A")
    f32 = fmt == "ts"
    S = 24 if f32 else 53
    rho = orc.rho(S, k)
    sl, ex = orc.split_plain(A, 1, "rows")
    for i in range(m):
        e = int(ex[0, i])
        for p in range(k):
            x = Fraction(float(A[0, p, i]))
            step = Fraction(2) ** (e + rho - S + (1 if x >= 0 else 0))
            q = x / step
            fl = math.floor(q)
            frac = q - fl
            nearest = fl + 1 if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2 == 1) else fl
            assert Fraction(float(sl[0, p, i])) == nearest * step


@pytest.mark.parametrize("fmt", ["dd", "qd", "ts"])
def test_literal_last_slice(orc, fmt):
    """Algorithm 1 as printed (last slice = leading component of the residual
    after D - 1 passes): the first D - 1 slices are those of the extracting
    split; slice D is the leading component of the (D - 1)-pass residual;
    slices plus the remaining residual still equal the input exactly; D = 1
    returns the input's leading components; and the independent Python split
    agrees bit for bit."""
    m, k, D = 6, 29, 5
    A = W.gen_matrix(fmt, m, k, E=16, seed=31, operand="A")
    f32 = fmt == "ts"
    lit, lex, lres = orc.split_plain(A, D, "rows", want_resid=True, last="remainder")
    ext, eex = orc.split_plain(A, D, "rows")
    _, _, res1 = orc.split_plain(A, D - 1, "rows", want_resid=True)
    assert np.array_equal(lit[: D - 1], ext[: D - 1]) and np.array_equal(lex, eex)
    assert np.array_equal(lit[D - 1], res1[0])
    for i in range(m):
        for p in range(k):
            tot = sum((Fraction(float(lit[a, p, i])) for a in range(D)), Fraction(0)) + X.value(lres[:, p, i])
            assert tot == X.value(A[:, p, i])
        vec = [tuple(A[:, p, i]) for p in range(k)]
        s2, _, _ = X.split_vector_py(vec, D, f32, last_remainder=True)
        for a in range(D):
            assert [float(v) for v in lit[a, :, i]] == [float(v) for v in s2[a]]
    one, _ = orc.split_plain(A, 1, "rows", last="remainder")
    assert np.array_equal(one[0], A[0])
    with pytest.raises(ValueError):
        orc.split_plain(A, D, "rows", last="rounded")


def test_zero_row_gives_zero_slices(orc):
    A = W.gen_matrix("dd", 4, 9, seed=1, operand="A")
    A[:, :, 2] = 0.0
    sl, ex = orc.split_plain(A, 3, "rows")
    assert np.all(sl[:, :, 2] == 0) and np.all(ex[:, 2] == orc.ZERO_EXP)
    assert np.all(ex[:, 0] != orc.ZERO_EXP)


def test_triangle_pairs_from_paper(orc):
    """The D = 3 product set of Section 3 (after Fig. 1): the oracle's C is the
    exact sum of exactly those slice products, and the count is D(D+1)/2."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "triangle_D3.txt")
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines[0] == ["D", "3"]
    pairs = {(int(a), int(b)) for a, b in lines[1:]}
    assert len(pairs) == 3 * 4 // 2
    m, n, k, D = 5, 4, 16, 3
    A, B = W.gen_pair("dd", m, n, k, E=4, seed=13)
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    rho = orc.rho(53, k)
    prods = {(a + 1, b + 1): orc.slice_product(sa[a], ea[a], sb[b], eb[b], rho, 53) for a in range(D) for b in range(D)}
    Ct, _ = orc.ozaki_gemm(A, B, D)
    for i in range(m):
        for j in range(n):
            want = orc.exact_sum([prods[p][j, i] for p in sorted(pairs)], 2)
            assert list(Ct[:, j, i]) == list(want)
    # the pairs outside the triangle are not negligible copies of zero
    assert any(np.any(prods[p] != 0) for p in [(2, 3), (3, 2), (3, 3)])
