"""CPU oracle for Ozaki-scheme multi-component GEMM (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps ``oracle.c`` (built by ``oracle/build.py``) and shares
no code with the HIP library.

Array conventions (the same as the product's Python binding): a matrix with
``rows`` rows and ``cols`` columns in a c-component format is a C-contiguous
array of shape ``(c, cols, rows)`` -- component-planar, each plane
column-major.  So A (m x k) is ``(c, k, m)``, B (k x n) is ``(c, n, k)`` and
C (m x n) is ``(c, n, m)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c (the sanitizer run of the oracle's tests)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
ZERO_EXP = -(2 ** 31)
C_OF = {"dd": 2, "td": 3, "qd": 4, "ts": 3}

_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_long


def lib():
    """The loaded oracle library (built first if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_two_sum.restype = ctypes.c_double
        L.oracle_two_sum.argtypes = [ctypes.c_double, ctypes.c_double, _P]
        L.oracle_two_sum_f.restype = ctypes.c_float
        L.oracle_two_sum_f.argtypes = [ctypes.c_float, ctypes.c_float, _P]
        L.oracle_two_prod.restype = ctypes.c_double
        L.oracle_two_prod.argtypes = [ctypes.c_double, ctypes.c_double, _P]
        L.oracle_renorm.argtypes = [_P, _I]
        L.oracle_renorm_f.argtypes = [_P, _I]
        L.oracle_rho.restype = _I
        L.oracle_rho.argtypes = [_I, _L]
        L.oracle_split_plain.argtypes = [_I, _I, _I, _P, _L, _L, _L, _I, _I, _I, _P, _P, _P]
        L.oracle_split_plain_f.argtypes = [_I, _I, _I, _P, _L, _L, _L, _I, _I, _I, _P, _P, _P]
        L.oracle_slice_product.argtypes = [_I, _I, _I, _P, _P, _P, _P, _I, _I, _P]
        L.oracle_gemm_exact_check.argtypes = [_I, _I, _I, _I, _I, _P, _P, _P, _I, _P, _I, _P, _P, _P]
        L.oracle_gemm_exact_check_many.argtypes = [_I, _I, _I, _I, _I, _P, _P, _I, _P, _I, _P, _I, _P, _P, _P]
        L.oracle_exact_sum.argtypes = [_P, _L, _I, _I, _P]
        L.oracle_ozaki_gemm.argtypes = [_I, _I, _I, _I, _I, _P, _P, _I, _P, _I, _P, _P]
        L.oracle_split_int8.argtypes = [_I, _I, _I, _P, _L, _L, _L, _I, _P, _P]
        L.oracle_int8_diag_sums.argtypes = [_I, _I, _I, _I, _P, _P, _P]
        L.oracle_int8_combine.argtypes = [_I, _I, _I, _I, _P, _P, _P, _P]
        L.oracle_gemm_naive.argtypes = [_I, _I, _I, _I, _I, _P, _P, _P, _I, _P]
        L.oracle_ds_round.argtypes = [_I, _L, _L, _P, _P, _P]
        L.oracle_gemm_naive_ds.argtypes = [_I, _I, _I, _P, _P, _P, _P, _P, _I, _P, _P]
        L.oracle_omp_threads.restype = _I
        L.oracle_set_threads.argtypes = [_I]
        L.oracle_set_threads.restype = _I
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(status, what):
    if status != 0:
        raise RuntimeError(f"oracle {what} failed with status {status}")


def set_threads(n: int) -> int:
    """Threads of the oracle's later parallel loops; returns the count in effect."""
    return int(lib().oracle_set_threads(int(n)))


def threads() -> int:
    return lib().oracle_omp_threads()


def two_sum(a: float, b: float):
    e = ctypes.c_double()
    s = lib().oracle_two_sum(a, b, ctypes.byref(e))
    return s, e.value


def two_sum_f(a, b):
    e = ctypes.c_float()
    s = lib().oracle_two_sum_f(float(a), float(b), ctypes.byref(e))
    return np.float32(s), np.float32(e.value)


def two_prod(a: float, b: float):
    e = ctypes.c_double()
    p = lib().oracle_two_prod(a, b, ctypes.byref(e))
    return p, e.value


def renorm(x) -> np.ndarray:
    x = np.array(x, dtype=np.float64 if np.asarray(x).dtype != np.float32 else np.float32)
    if x.dtype == np.float32:
        lib().oracle_renorm_f(_ptr(x), len(x))
    else:
        lib().oracle_renorm(_ptr(x), len(x))
    return x


def rho(S: int, k: int) -> int:
    """The shift ceil((S + log2 k)/2) of Algorithm 1 (Section 3)."""
    return lib().oracle_rho(S, k)


def _split_axes(X, along):
    c, cols, rows = X.shape
    if along == "rows":  # rows of a (rows x cols) matrix: vectors are rows, length cols
        return rows, cols, 1, rows, rows * cols
    if along == "cols":
        return cols, rows, rows, 1, rows * cols
    raise ValueError(along)


def split_plain(X: np.ndarray, D: int, along: str, *, want_resid: bool = False, last: str = "extract"):
    """Algorithm 1's split of every row (``along='rows'``, operand A) or column
    (``along='cols'``, operand B) of X (shape ``(c, cols, rows)``).

    Returns ``(slices, exps[, resid])``: slices ``(D, cols, rows)`` in X's
    dtype, exps ``(D, nvec)`` int32 holding ceil(log2 mu) per pass (ZERO_EXP
    when mu = 0), resid ``(c, cols, rows)`` the remainder after D passes.

    ``last='extract'``: D slices on the grid of tau, remainder dropped (every
    slice product exact).  ``last='remainder'``: Algorithm 1 as printed, the
    D-th slice is the leading component of the residual after D - 1 passes.
    """
    if last not in ("extract", "remainder"):
        raise ValueError(last)
    X = np.ascontiguousarray(X)
    c = X.shape[0]
    nvec, ln, s_vec, s_elt, s_comp = _split_axes(X, along)
    f32 = X.dtype == np.float32
    S = 24 if f32 else 53
    r = rho(S, ln)
    slices = np.zeros((D,) + X.shape[1:], dtype=X.dtype)
    exps = np.zeros((D, nvec), dtype=np.int32)
    resid = np.zeros_like(X) if want_resid else None
    fn = lib().oracle_split_plain_f if f32 else lib().oracle_split_plain
    _check(fn(nvec, ln, c, _ptr(X), s_vec, s_elt, s_comp, D, r, 1 if last == "remainder" else 0, _ptr(slices),
              _ptr(exps), _ptr(resid)), "split")
    return (slices, exps, resid) if want_resid else (slices, exps)


def slice_product(Aa, ea, Bb, eb, k_rho: int, S: int) -> np.ndarray:
    """Exact C_ab = A_a B_b (Section 3): Aa ``(k, m)``, Bb ``(n, k)`` -> ``(n, m)`` float64."""
    Aa = np.ascontiguousarray(Aa, dtype=np.float64)
    Bb = np.ascontiguousarray(Bb, dtype=np.float64)
    ea = np.ascontiguousarray(ea, dtype=np.int32)
    eb = np.ascontiguousarray(eb, dtype=np.int32)
    k, m = Aa.shape
    n = Bb.shape[0]
    out = np.zeros((n, m), dtype=np.float64)
    _check(lib().oracle_slice_product(m, n, k, _ptr(Aa), _ptr(ea), _ptr(Bb), _ptr(eb), k_rho, S, _ptr(out)),
           "slice_product")
    return out


def exact_check(A, B, C, rows=None):
    """Exact comparison of ``C`` with ``A B`` for the given rows of C.

    Returns ``(diff, absab, cex)``, each ``(n, nrows)`` float64: ``|C - AB|``
    rounded once, ``sum_p |a_ip||b_pj|`` from leading components, and ``AB``
    rounded once.
    """
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    C = np.ascontiguousarray(C)
    c, k, m = A.shape
    n = B.shape[1]
    f32 = A.dtype == np.float32
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nrows = m if rows is None else len(rows_arr)
    ldc = C.shape[2]
    diff = np.zeros((n, nrows))
    absab = np.zeros((n, nrows))
    cex = np.zeros((n, nrows))
    _check(lib().oracle_gemm_exact_check(c, int(f32), m, n, k, _ptr(A), _ptr(B), _ptr(C), ldc, _ptr(rows_arr),
                                         nrows, _ptr(diff), _ptr(absab), _ptr(cex)), "exact_check")
    return diff, absab, cex


def exact_check_many(A, B, Cs, rows=None):
    """``exact_check`` of several results of the same product at once: the
    exact AB of each listed entry is formed once and compared with every C in
    ``Cs`` (all of one shape).  Returns ``(diffs, absab, cex)`` with diffs a
    list of ``(n, nrows)`` arrays, one per C."""
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    Cs = [np.ascontiguousarray(C) for C in Cs]
    c, k, m = A.shape
    n = B.shape[1]
    f32 = A.dtype == np.float32
    if any(C.shape != Cs[0].shape or C.dtype != A.dtype for C in Cs):
        raise ValueError("every C must have one shape and the dtype of A")
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nrows = m if rows is None else len(rows_arr)
    ldc = Cs[0].shape[2]
    diff = np.zeros((len(Cs), n, nrows))
    absab = np.zeros((n, nrows))
    cex = np.zeros((n, nrows))
    ptrs = (ctypes.c_void_p * max(1, len(Cs)))(*[C.ctypes.data for C in Cs])
    _check(lib().oracle_gemm_exact_check_many(c, int(f32), m, n, k, _ptr(A), _ptr(B), len(Cs), ptrs, ldc,
                                              _ptr(rows_arr), nrows, _ptr(diff), _ptr(absab), _ptr(cex)),
           "exact_check_many")
    return list(diff), absab, cex


def exact_sum(values, c: int, f32: bool = False) -> np.ndarray:
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.zeros(c)
    _check(lib().oracle_exact_sum(_ptr(v), len(v), c, int(f32), _ptr(out)), "exact_sum")
    return out


def ozaki_gemm(A, B, D: int, rows=None, paper: bool = False):
    """Ozaki product (Algorithm 1) of A ``(c, k, m)`` and B ``(c, n, k)``.

    Returns ``(C_tri, C_paper)``: ``(c, n, nrows)`` float64 arrays (components
    of TS results are binary32 values stored as float64); ``C_paper`` is None
    unless ``paper``.
    """
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    c, k, m = A.shape
    n = B.shape[1]
    f32 = A.dtype == np.float32
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nrows = m if rows is None else len(rows_arr)
    C_tri = np.zeros((c, n, nrows))
    C_pap = np.zeros((c, n, nrows)) if paper else None
    _check(lib().oracle_ozaki_gemm(c, int(f32), m, n, k, _ptr(A), _ptr(B), D, _ptr(rows_arr), nrows, _ptr(C_tri),
                                   _ptr(C_pap)), "ozaki_gemm")
    return C_tri, C_pap


def split_int8(X: np.ndarray, D: int, along: str):
    """INT8 digit planes ``(D, cols, rows)`` int8 and exponents E ``(nvec,)``."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    c = X.shape[0]
    nvec, ln, s_vec, s_elt, s_comp = _split_axes(X, along)
    digits = np.zeros((D,) + X.shape[1:], dtype=np.int8)
    exps = np.zeros(nvec, dtype=np.int32)
    _check(lib().oracle_split_int8(nvec, ln, c, _ptr(X), s_vec, s_elt, s_comp, D, _ptr(digits), _ptr(exps)),
           "split_int8")
    return digits, exps


def int8_diag_sums(Ad, Bd) -> np.ndarray:
    """S_g = sum_{s+t=g+1} A_s B_t for g = 1..D: ``(D, n, m)`` int64."""
    Ad = np.ascontiguousarray(Ad, dtype=np.int8)
    Bd = np.ascontiguousarray(Bd, dtype=np.int8)
    D, k, m = Ad.shape
    n = Bd.shape[1]
    S = np.zeros((D, n, m), dtype=np.int64)
    _check(lib().oracle_int8_diag_sums(m, n, k, D, _ptr(Ad), _ptr(Bd), _ptr(S)), "int8_diag_sums")
    return S


def int8_combine(S, EA, EB, c: int) -> np.ndarray:
    S = np.ascontiguousarray(S, dtype=np.int64)
    EA = np.ascontiguousarray(EA, dtype=np.int32)
    EB = np.ascontiguousarray(EB, dtype=np.int32)
    D, n, m = S.shape
    C = np.zeros((c, n, m))
    _check(lib().oracle_int8_combine(m, n, D, c, _ptr(S), _ptr(EA), _ptr(EB), _ptr(C)), "int8_combine")
    return C


def int8_gemm(A, B, D: int):
    """INT8-form product: split, diagonal sums, exact combination."""
    Ad, EA = split_int8(A, D, "rows")
    Bd, EB = split_int8(B, D, "cols")
    S = int8_diag_sums(Ad, Bd)
    return int8_combine(S, EA, EB, A.shape[0])


def gemm_naive(A, B, rows=None) -> np.ndarray:
    """The paper's simple triple-loop product in the multi-component format."""
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    c, k, m = A.shape
    n = B.shape[1]
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nrows = m if rows is None else len(rows_arr)
    C = np.zeros((c, n, nrows), dtype=A.dtype)
    _check(lib().oracle_gemm_naive(c, int(A.dtype == np.float32), m, n, k, _ptr(A), _ptr(B), _ptr(rows_arr), nrows,
                                   _ptr(C)), "gemm_naive")
    return C


def ds_round(X):
    """D+S rounding of exact sums: X ``(c, ...)`` float64 component planes;
    returns ``(hi, lo)`` with the shape of one plane, hi = RN53(sum) (float64)
    and lo = RN24(sum - hi) (float32), from the exact value."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    c = X.shape[0]
    count = X[0].size
    hi = np.zeros(X.shape[1:], dtype=np.float64)
    lo = np.zeros(X.shape[1:], dtype=np.float32)
    _check(lib().oracle_ds_round(c, count, count, _ptr(X), _ptr(hi), _ptr(lo)), "ds_round")
    return hi, lo


def gemm_naive_ds(Ahi, Alo, Bhi, Blo, rows=None):
    """The simple triple loop in D+S (DD arithmetic on the exact DD reading of
    each D+S input, C rounded to D+S once).  Inputs as ``workload.gen_ds``:
    ``(1, k, m)`` / ``(1, n, k)`` planes.  Returns ``(Chi, Clo)`` of shape
    ``(1, n, nrows)``."""
    Ahi, Bhi = np.ascontiguousarray(Ahi, dtype=np.float64), np.ascontiguousarray(Bhi, dtype=np.float64)
    Alo, Blo = np.ascontiguousarray(Alo, dtype=np.float32), np.ascontiguousarray(Blo, dtype=np.float32)
    _, k, m = Ahi.shape
    n = Bhi.shape[1]
    rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nrows = m if rows is None else len(rows_arr)
    Chi = np.zeros((1, n, nrows), dtype=np.float64)
    Clo = np.zeros((1, n, nrows), dtype=np.float32)
    _check(lib().oracle_gemm_naive_ds(m, n, k, _ptr(Ahi), _ptr(Alo), _ptr(Bhi), _ptr(Blo), _ptr(rows_arr), nrows,
                                      _ptr(Chi), _ptr(Clo)), "gemm_naive_ds")
    return Chi, Clo


def ds_as_dd(hi, lo):
    """A D+S array pair as a two-component binary64 array (exact)."""
    return np.concatenate([np.asarray(hi, dtype=np.float64), np.asarray(lo, dtype=np.float64)], axis=0)


def bound_report(diff, absab, t: int):
    """Elementwise bound ``|C - AB| <= 2^-t (|A||B|)``.

    ``absab`` is computed from leading components, so it is within a relative
    (k + 2) 2^-52 of the true value; the check allows that slack.  Returns
    ``(ok, worst_log2_ratio)`` where the ratio is ``diff / absab`` (an element
    with ``absab == 0`` must have ``diff == 0``).
    """
    diff = np.asarray(diff)
    absab = np.asarray(absab)
    zero = absab == 0
    if np.any(diff[zero] != 0):
        return False, float("inf")
    nz = ~zero
    if not np.any(nz):
        return True, float("-inf")
    ratio = diff[nz] / absab[nz]
    worst = float(np.max(ratio))
    ok = bool(np.all(diff[nz] <= np.ldexp(absab[nz], -t) * (1 + 2.0 ** -30)))
    return ok, (float(np.log2(worst)) if worst > 0 else float("-inf"))


def certificate_terms(A, B, D: int, form: str = "float", pairs=None):
    """The truncation part of the a-posteriori error bound of the D-slice
    product (Algorithm 1 and the pairs a + b <= D + 1 of Section 3), in exact
    rational arithmetic (small inputs only).  ``form='int8'``: the slices are
    the INT8 digit planes, slice s of vector v being d_s 2^(E_v - 6 - 7 (s - 1))
    with |d_s| <= 64, so it is bounded by 2^(E_v - 7 (s - 1)), and the remainder
    after D digits by 2^(E_v - 7 D) (1 + 2^-40).

    With A = A_s + RA and B = B_s + RB (slices plus the remainder of the D
    passes), AB - C_tri = (pairs a + b > D + 1) + A_s RB + RA B.  Per entry:
      T1 = k sum over the left-out pairs of 2^(eA_a,i + eB_b,j)   (|A_a| <= 2^eA_a)
      T2 = rB_j (sum_p |a_ip| + k rA_i),  T3 = rA_i sum_p |b_pj|,
    rA_i = 2^(eA_D,i + rho - S) (1 + 2^(1 - rho)) bounding the remainder.
    Returns ``(trunc, T1, T23, absab)`` as lists ``[i][j]`` of Fractions: the
    exact |C_tri - AB| from this oracle's slices, T1, T2 + T3, and (|A||B|)_ij.

    ``pairs(i, j)``: another pair set per entry instead of the triangle, given
    as D counts (0-based slice a of A pairs with slices b < counts[a] of B);
    C_tri is then the sum over that set, and T1 runs over every other pair.
    """
    from fractions import Fraction

    from . import exact as X
    f32 = A.dtype == np.float32
    S = 24 if f32 else 53
    c, k, m = A.shape
    n = B.shape[1]
    r = rho(S, k)

    def p2(e):
        return Fraction(2) ** int(e)

    Av = X.matrix_values(A)  # Av[i][p]
    Bv = X.matrix_values(B)  # Bv[p][j]
    if form == "int8":
        da, EA = split_int8(A, D, "rows")
        db, EB = split_int8(B, D, "cols")

        def unit(E, s):
            return p2(E - 6 - 7 * s)  # 0-based digit s

        SA = [[[0 if EA[i] == ZERO_EXP else int(da[a, p, i]) * unit(EA[i], a) for p in range(k)] for i in range(m)]
              for a in range(D)]
        SB = [[[0 if EB[j] == ZERO_EXP else int(db[b, j, p]) * unit(EB[j], b) for p in range(k)] for j in range(n)]
              for b in range(D)]
        ea = np.array([[ZERO_EXP if E == ZERO_EXP else E - 7 * a for E in EA] for a in range(D)], dtype=np.int64)
        eb = np.array([[ZERO_EXP if E == ZERO_EXP else E - 7 * b for E in EB] for b in range(D)], dtype=np.int64)
        margin = 1 + Fraction(2) ** -40
        rA = [0 if EA[i] == ZERO_EXP else p2(EA[i] - 7 * D) * margin for i in range(m)]
        rB = [0 if EB[j] == ZERO_EXP else p2(EB[j] - 7 * D) * margin for j in range(n)]
    else:
        sa, ea = split_plain(A, D, "rows")
        sb, eb = split_plain(B, D, "cols")
        SA = [[[Fraction(float(sa[a, p, i])) for p in range(k)] for i in range(m)] for a in range(D)]
        SB = [[[Fraction(float(sb[b, j, p])) for p in range(k)] for j in range(n)] for b in range(D)]
        rem = 1 + Fraction(2) ** (1 - r)
        rA = [0 if ea[D - 1, i] == ZERO_EXP else p2(ea[D - 1, i] + r - S) * rem for i in range(m)]
        rB = [0 if eb[D - 1, j] == ZERO_EXP else p2(eb[D - 1, j] + r - S) * rem for j in range(n)]
    rs = [sum((abs(Av[i][p]) for p in range(k)), Fraction(0)) for i in range(m)]
    cs = [sum((abs(Bv[p][j]) for p in range(k)), Fraction(0)) for j in range(n)]
    trunc, T1, T23, absab = [], [], [], []
    for i in range(m):
        tr, t1s, t23s, ab = [], [], [], []
        for j in range(n):
            exact = sum((Av[i][p] * Bv[p][j] for p in range(k)), Fraction(0))
            # 0-based a + b <= D - 1 (1-based a + b <= D + 1), or the given set
            counts = [D - a for a in range(D)] if pairs is None else list(pairs(i, j))
            ctri = Fraction(0)
            t1 = Fraction(0)
            for a in range(D):
                for b in range(D):
                    if b < counts[a]:
                        ctri += sum((SA[a][i][p] * SB[b][j][p] for p in range(k)), Fraction(0))
                    elif ea[a, i] != ZERO_EXP and eb[b, j] != ZERO_EXP:
                        t1 += p2(ea[a, i] + eb[b, j])
            t1s.append(t1 * k)
            t23s.append(rB[j] * (rs[i] + k * rA[i]) + rA[i] * cs[j])
            tr.append(abs(ctri - exact))
            ab.append(sum((abs(Av[i][p] * Bv[p][j]) for p in range(k)), Fraction(0)))
        trunc.append(tr)
        T1.append(t1s)
        T23.append(t23s)
        absab.append(ab)
    return trunc, T1, T23, absab
