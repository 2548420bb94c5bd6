"""Pins of the oracle's products and its Ozaki GEMM against exact rational /
integer arithmetic, closed forms and special cases that reduce to a textbook
result."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle.exact as X
import workload as W
from digit_cases import tie_cases

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}


def _formats():
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_formats.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, c, cb, L = line.split()
            out[name] = (int(c), int(cb), int(L))
    return out


def test_formats_match_paper_lengths():
    """c components of cb bits give the paper's L bits (Sections 1 and 4.4), and
    the error-bound exponents sit below L."""
    f = _formats()
    for name, (c, cb, L) in f.items():
        assert c * cb == L
        assert T_BITS[name] < L
        assert W.FORMATS[name][0] == c


@pytest.mark.parametrize("fmt", ["dd", "td", "qd", "ts"])
def test_exact_check_against_fractions(orc, fmt):
    m, n, k = 3, 4, 6
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=4)
    C = np.zeros((A.shape[0], n, m), dtype=A.dtype)
    C[0] = 1.0
    Cf = X.matmul_fraction(A, B)
    diff, absab, cex = orc.exact_check(A, B, C)
    for i in range(m):
        for j in range(n):
            assert cex[j, i] == float(Cf[i][j])
            assert diff[j, i] == float(abs(Fraction(1) - Cf[i][j]))
            ab = sum(abs(Fraction(float(A[0, p, i]))) * abs(Fraction(float(B[0, j, p]))) for p in range(k))
            assert abs(Fraction(absab[j, i]) - ab) <= ab * Fraction(2) ** -48


@pytest.mark.parametrize("fmt", ["dd", "qd", "ts"])
def test_exact_check_many_against_fractions(orc, fmt):
    """Several results compared with one exact product: each difference equals
    the rational |C_u - AB| rounded once, on a subset of rows (the row index
    must map to the right row of every C), and an exactly rounded C_u gives
    the rational rounding error of its own components."""
    m, n, k = 5, 3, 7
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=9)
    c = A.shape[0]
    Cf = X.matmul_fraction(A, B)
    Cs = []
    for u in range(3):
        C = np.zeros((c, n, m), dtype=A.dtype)
        for i in range(m):
            for j in range(n):
                C[0, j, i] = float(Cf[i][j]) * (1 + u * 2.0 ** -20) + u * (i - j)
                if c > 1 and u == 1:
                    C[1, j, i] = 2.0 ** -30 * (i + 1)
        Cs.append(C)
    rows = [4, 0, 2]
    diffs, absab, cex = orc.exact_check_many(A, B, Cs, rows=rows)
    assert len(diffs) == 3
    for u, C in enumerate(Cs):
        for t, i in enumerate(rows):
            for j in range(n):
                got = sum(Fraction(float(C[r, j, i])) for r in range(c))
                assert diffs[u][j, t] == float(abs(got - Cf[i][j])), (u, i, j)
                assert cex[j, t] == float(Cf[i][j])
    # the same arrays as the single-matrix form, entry for entry
    for u, C in enumerate(Cs):
        d1, a1, _ = orc.exact_check(A, B, C, rows=rows)
        assert np.array_equal(d1, diffs[u]) and np.array_equal(a1, absab)


def test_slice_product_exact_non_square(orc):
    """C_ab from exact int64 dot products equals the rational product (a 5x3 times 3x7
    shape, so a transposed operand cannot pass)."""
    m, n, k, D = 5, 7, 3, 3
    A, B = W.gen_pair("td", m, n, k, E=8, seed=8)
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    rho = orc.rho(53, k)
    for a in range(D):
        for b in range(D):
            P = orc.slice_product(sa[a], ea[a], sb[b], eb[b], rho, 53)
            for i in range(m):
                for j in range(n):
                    want = sum(Fraction(float(sa[a, p, i])) * Fraction(float(sb[b, j, p])) for p in range(k))
                    assert Fraction(P[j, i]) == want


def test_config0_dd_128_meets_bound_against_python_integers(orc):
    """DD, m = n = k = 128, e ~ U{0..8}: the oracle's Ozaki C (D = 6) is within
    2^-100 |A||B| of the exact product computed by Python integers."""
    m = n = k = 128
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=0)
    C, Cp = orc.ozaki_gemm(A, B, 6, paper=True)
    Cint, q = X.matmul_exact_int(A, B)
    absA = np.abs(A[0]).T  # (m, k)
    absB = np.abs(B[0]).T  # (k, n)
    absab = absA @ absB
    worst = -1e9
    for Cx in (C, Cp):
        for i in range(0, m, 3):
            for j in range(n):
                exact = Fraction(Cint[i][j]) * Fraction(2) ** q
                err = abs(X.value(Cx[:, j, i]) - exact)
                bound = Fraction(float(absab[i, j])) * Fraction(2) ** -100 * (1 + Fraction(2) ** -30)
                assert err <= bound, (i, j)
                if err:
                    worst = max(worst, float(np.log2(float(err / Fraction(float(absab[i, j]))))))
    assert worst < -100
    # the C exact check agrees with the Python integers on a sample
    diff, _, cex = orc.exact_check(A, B, C, rows=[0, 77])
    for t, i in enumerate([0, 77]):
        for j in range(0, n, 17):
            exact = Fraction(Cint[i][j]) * Fraction(2) ** q
            assert cex[j, t] == float(exact)
            assert diff[j, t] == float(abs(X.value(C[:, j, i]) - exact))


@pytest.mark.parametrize("fmt,D", [("dd", 6), ("td", 9), ("qd", 11), ("ts", 13)])
def test_ozaki_meets_bound_ragged(orc, fmt, D):
    m, n, k = 33, 21, 300
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=17)
    C, Cp = orc.ozaki_gemm(A, B, D, paper=True)
    for Cx in (C, Cp):
        diff, absab, _ = orc.exact_check(A, B, Cx.astype(A.dtype))
        ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
        assert ok, worst


def test_dropping_a_term_breaks_the_bound(orc):
    """The bound has teeth: with D = 5 at k = 64 the full triangle meets
    2^-100 |A||B|, and leaving out one of its slice products (the pair (1, D))
    does not."""
    m, n, k, D = 8, 8, 64, 5
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=3)
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    rho = orc.rho(53, k)
    full = np.zeros((2, n, m))
    dropped = np.zeros((2, n, m))
    for i in range(m):
        for j in range(n):
            terms = {}
            for a in range(D):
                for b in range(D - a):
                    terms[(a, b)] = orc.slice_product(sa[a][:, i:i + 1], ea[a][i:i + 1], sb[b][j:j + 1],
                                                      eb[b][j:j + 1], rho, 53)[0, 0]
            full[:, j, i] = orc.exact_sum(list(terms.values()), 2)
            dropped[:, j, i] = orc.exact_sum([v for key, v in terms.items() if key != (0, D - 1)], 2)
    diff, absab, _ = orc.exact_check(A, B, full)
    assert orc.bound_report(diff, absab, 100)[0]
    diff, absab, _ = orc.exact_check(A, B, dropped)
    ok, worst = orc.bound_report(diff, absab, 100)
    assert not ok and worst > -100


def test_identity_gives_input(orc):
    """B = I with enough slices to exhaust A: C is A's exact value (as its
    canonical greedy expansion)."""
    m, k = 9, 12
    A = W.gen_matrix("dd", m, k, E=4, seed=6, operand="A")
    B = np.zeros((2, k, k))
    B[0] = np.eye(k)
    C, _ = orc.ozaki_gemm(A, B, 12)
    for i in range(m):
        for j in range(k):
            assert list(C[:, j, i]) == list(orc.exact_sum(list(A[:, j, i]), 2))


def test_single_slice_is_one_exact_product(orc):
    m, n, k = 6, 5, 40
    A, B = W.gen_pair("qd", m, n, k, E=8, seed=2)
    sa, ea = orc.split_plain(A, 1, "rows")
    sb, eb = orc.split_plain(B, 1, "cols")
    P = orc.slice_product(sa[0], ea[0], sb[0], eb[0], orc.rho(53, k), 53)
    C, _ = orc.ozaki_gemm(A, B, 1)
    assert np.array_equal(C[0], P) and np.all(C[1:] == 0)


def test_zero_and_small_integers(orc):
    m, n, k = 7, 6, 50
    A = np.zeros((2, k, m))
    B = W.gen_matrix("dd", k, n, seed=1, operand="B")
    C, _ = orc.ozaki_gemm(A, B, 4)
    assert np.all(C == 0)
    rng = np.random.default_rng(0)
    Ai = rng.integers(-1023, 1024, size=(m, k))
    Bi = rng.integers(-1023, 1024, size=(k, n))
    A = np.zeros((2, k, m))
    B = np.zeros((2, n, k))
    A[0] = Ai.T
    B[0] = Bi.T
    C, _ = orc.ozaki_gemm(A, B, 3)
    ref = Ai @ Bi  # exact in int64
    assert np.array_equal(C[0], ref.T.astype(np.float64)) and np.all(C[1] == 0)


def test_power_of_two_scaling_is_exact(orc):
    m, n, k, D = 6, 5, 33, 5
    A, B = W.gen_pair("td", m, n, k, E=8, seed=12)
    C, _ = orc.ozaki_gemm(A, B, D)
    A2 = A.copy()
    A2[:, :, 3] *= 2.0 ** 37
    B2 = B.copy()
    B2[:, 2, :] *= 2.0 ** -21
    C2, _ = orc.ozaki_gemm(A2, B2, D)
    expect = C.copy()
    expect[:, :, 3] *= 2.0 ** 37
    expect[:, 2, :] *= 2.0 ** -21
    assert np.array_equal(C2, expect)


def test_error_falls_with_D_and_saturates_on_eq1_data(orc):
    """Paper trend (Section 4.1): on eq. (1) matrices the DD error falls as D
    grows and stops improving around D = 6 (at the DD rounding level)."""
    m = n = k = 64
    A, B = W.gen_pair("dd", m, n, k, seed=1, spread="eq1")
    errs = []
    for D in range(2, 9):
        C, _ = orc.ozaki_gemm(A, B, D)
        diff, absab, cex = orc.exact_check(A, B, C)
        rel = np.max(diff / np.maximum(np.abs(cex), 1e-300))  # the paper's max relative error
        errs.append(np.log2(rel))
    assert all(errs[i + 1] < errs[i] - 10 for i in range(3))  # D = 2..5 each gain > 10 bits
    assert abs(errs[-1] - errs[-3]) < 6 and errs[-1] < -95  # D = 6..8 saturate near 2^-106


@pytest.mark.parametrize("fmt,D", [("dd", 17), ("qd", 17), ("8d", 61), ("14d", 104)])
def test_int8_digits_against_python_rationals(orc, fmt, D):
    """INT8 digits: equal to an independent rational implementation of the same
    rule; |d| <= 64; and the closed form: for every s, sum_{t <= s} d_t u_t is
    x rounded to nearest (ties to even) on the grid u_s, so the remainder after
    D digits is at most u_D / 2.  Long expansions (8 and 14 binary64
    components) included."""
    m, k = 4, 9
    A = W.gen_matrix(fmt, m, k, E=16, seed=31, operand="A")
    dg, E = orc.split_int8(A, D, "rows")
    for i in range(m):
        want, Ew = X.int8_digits_py([tuple(A[:, p, i]) for p in range(k)], D)
        assert E[i] == Ew
        for p in range(k):
            assert list(dg[:, p, i]) == want[p]
            check_digit_closed_form(A[:, p, i], dg[:, p, i], int(E[i]))


def check_digit_closed_form(comps, digits, E):
    x = X.value(comps)
    partial = Fraction(0)
    for s, d in enumerate(digits, start=1):
        assert -64 <= int(d) <= 64
        u = Fraction(2) ** (E - 6 - 7 * (s - 1))
        partial += int(d) * u
        assert partial == X.rne(x / u) * u, (s, comps)
    assert abs(x - partial) <= u / 2


@pytest.mark.parametrize("c,D", [(2, 17), (3, 24), (4, 31), (8, 61)])
def test_int8_digits_on_rounding_boundaries(orc, c, D):
    """Exact ties and near-ties at every level: the digits follow the exact
    value (a tie moved by 2^-70 of a unit rounds away from it; an exact tie
    goes to the even neighbour), as the rational implementation and the closed
    form say."""
    E = 3
    cases = tie_cases(c, D, E, seed=c)
    k = len(cases)
    A = np.zeros((c, k, 1))
    for p, comps in enumerate(cases):
        A[:, p, 0] = comps
    dg, Eo = orc.split_int8(A, D, "rows")
    assert Eo[0] == E
    want, _ = X.int8_digits_py([tuple(A[:, p, 0]) for p in range(k)], D)
    for p in range(k):
        assert list(dg[:, p, 0]) == want[p], cases[p]
        check_digit_closed_form(A[:, p, 0], dg[:, p, 0], E)


def test_int8_diag_sums_and_combination(orc):
    m, n, k, D = 5, 4, 7, 6
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=5)
    Ad, EA = orc.split_int8(A, D, "rows")
    Bd, EB = orc.split_int8(B, D, "cols")
    S = orc.int8_diag_sums(Ad, Bd)
    Ai = Ad.astype(np.int64)
    Bi = Bd.astype(np.int64)
    for g in range(1, D + 1):
        ref = np.zeros((n, m), dtype=np.int64)
        for s in range(1, g + 1):
            t = g + 1 - s
            ref += (Ai[s - 1].T @ Bi[t - 1].T).T  # (m,k)@(k,n) -> (m,n) -> (n,m)
        assert np.array_equal(S[g - 1], ref)
    C = orc.int8_combine(S, EA, EB, 2)
    for i in range(m):
        for j in range(n):
            v = sum(Fraction(int(S[g - 1, j, i])) * Fraction(2) ** (int(EA[i]) + int(EB[j]) + 2 - 7 * (g + 1))
                    for g in range(1, D + 1))
            assert C[0, j, i] == float(v) and C[1, j, i] == float(v - Fraction(C[0, j, i]))


@pytest.mark.parametrize("fmt,D", [("dd", 17), ("td", 24), ("qd", 31), ("6d", 46), ("10d", 74), ("14d", 103)])
def test_int8_form_meets_bound(orc, fmt, D):
    """INT8 form within 2^-t (|A||B|), t = 50 c (100 / 150 / 200 for DD / TD / QD)."""
    m, n, k = 19, 13, 200 if fmt in T_BITS else 60
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=23)
    C = orc.int8_gemm(A, B, D)
    diff, absab, _ = orc.exact_check(A, B, C)
    t = T_BITS.get(fmt, 50 * A.shape[0])
    ok, worst = orc.bound_report(diff, absab, t)
    assert ok, worst
    if fmt not in T_BITS:  # the last digits matter: four fewer miss the bound
        C4 = orc.int8_gemm(A, B, D - 4)
        diff4, _, _ = orc.exact_check(A, B, C4)
        assert not orc.bound_report(diff4, absab, t)[0]


@pytest.mark.parametrize("fmt", ["8d", "14d"])
def test_exact_check_long_expansions(orc, fmt):
    """The exact checker with 8 and 14 components: AB rounded once equals the
    rational product rounded, and C = that rounding's greedy expansion has
    |C - AB| below 2^-(53 c - 1) |AB|."""
    m, n, k = 3, 2, 4
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=41)
    c = A.shape[0]
    P = X.matmul_fraction(A, B)  # (m, n) exact
    C = np.zeros((c, n, m))
    for i in range(m):
        for j in range(n):
            r = P[i][j]
            for q in range(c):  # greedy expansion of the exact value
                C[q, j, i] = float(r)
                r -= Fraction(C[q, j, i])
    diff, absab, cex = orc.exact_check(A, B, C)
    for i in range(m):
        for j in range(n):
            assert cex[j, i] == float(P[i][j])
            assert diff[j, i] <= abs(float(P[i][j])) * 2.0 ** -(53 * c - 1)


@pytest.mark.parametrize("fmt", ["dd", "td", "qd", "ts"])
def test_naive_loop_accuracy(orc, fmt):
    """The paper's simple triple loop (Section 4.1) is accurate to about
    k 2^-(L-2) |A||B| (checked exactly)."""
    m, n, k = 6, 5, 32
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=9)
    C = orc.gemm_naive(A, B)
    diff, absab, _ = orc.exact_check(A, B, C)
    L = {"dd": 106, "td": 159, "qd": 212, "ts": 72}[fmt]
    assert np.all(diff <= absab * k * 2.0 ** -(L - 3))


def test_exponent_spread_beyond_the_automatic_slice_count(orc):
    """Algorithm 1 at a fixed D loses accuracy when one row of A and one
    column of B hold entries 2^40 apart that meet in the product (the slice
    grid is set by the row's and column's largest entry): DD with k = 2,
    A's row [x, 2^-40 u] and B's column [2^-40 v, y], all full-precision DD
    values.  D = 5 (the a-priori count for k = 2) misses 2^-100 |A||B|; D = 6
    meets it.  This is the case the automatic D does not cover and the
    certificate or the data-chosen pair sets handle."""
    rng = np.random.default_rng(5)

    def dd(scale):
        hi = rng.uniform(1.0, 2.0) * scale
        return hi, hi * 2.0 ** -53 * rng.uniform(-0.5, 0.5)

    worst5, worst6 = [], []
    for _ in range(8):
        A = np.zeros((2, 2, 1))
        B = np.zeros((2, 1, 2))
        A[:, 0, 0], A[:, 1, 0] = dd(1.0), dd(2.0 ** -40)
        B[:, 0, 0], B[:, 0, 1] = dd(2.0 ** -40), dd(1.0)
        for D, out in ((5, worst5), (6, worst6)):
            C, _ = orc.ozaki_gemm(A, B, D)
            diff, absab, _ = orc.exact_check(A, B, C)
            out.append(orc.bound_report(diff, absab, 100)[1])
    assert max(worst5) > -100  # the bound is missed at D = 5
    assert max(worst6) <= -100  # and met at D = 6
