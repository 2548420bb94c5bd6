"""Seeded synthetic inputs for multi-component GEMM, shared by the oracle and
the GPU path.

This module holds input generation only: no step of the splitting, slice
products or accumulation lives here.  Every value is a deterministic function
of ``(seed, operand, draw, element index)`` through a counter-based generator,
so any process (CPU test, GPU test, benchmark) reproduces identical bits.

Recipe (synthetic stand-in for the paper's random test matrices of Section 1,
eq. (1), which draw ``(ru - 0.5) * exp(rn)``; here the exponent spread is a
uniform integer instead of a log-normal factor, so the spread is a parameter):

* binary64 formats (DD, TD, QD with c = 2, 3, 4 components; "5d" .. "14d"
  with c = 5 .. 14):
  ``x0 = u * 2**e`` with ``u`` uniform on ``[-1, 1)`` on a ``2**-52`` grid and
  ``e`` a uniform integer in ``{0..E}``; then
  ``x_r = RN(x_{r-1} * 2**-53 * v_r)`` with ``v_r`` uniform on ``[-0.5, 0.5)``,
  so ``|x_r| <= 2**-54 |x_{r-1}| < ulp(x_{r-1}) / 2`` (a normalized expansion).
* TS (c = 3 binary32 components): the same with a ``2**-23`` grid for ``u``
  and ``x_r = RN_f32(x_{r-1} * 2**-24 * v_r)``.
* D+S (``gen_ds``): the DD leading component with the second component
  rounded to binary32.
* ``eq1`` spread: ``x0 = (ru - 0.5) * exp(rn)`` with ``ru`` uniform on
  ``[0, 1)`` and ``rn`` standard normal (Box-Muller on two uniforms), the
  paper's own distribution, with lower components drawn as above.

Layout: a matrix of ``rows x cols`` is returned as a C-contiguous array of
shape ``(c, cols, rows)``: component-planar, each plane column-major with
leading dimension ``rows``.
"""
from __future__ import annotations

import numpy as np

FORMATS = {"dd": (2, np.float64), "td": (3, np.float64), "qd": (4, np.float64), "ts": (3, np.float32)}
# longer binary64 expansions ("5d" .. "14d": 265 to 742 bits in 53-bit steps)
FORMATS.update({f"{c}d": (c, np.float64) for c in range(5, 15)})

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_OPERANDS = {"A": 1, "B": 2}


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea, Flood 2014) on uint64 arrays."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _stream_key(seed: int, operand: int, draw: int) -> np.uint64:
    k = np.array([(seed * 1_000_003 + operand * 7919 + draw * 104_729) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(k)[0]


def random_u64(seed: int, operand: int, draw: int, count: int) -> np.ndarray:
    """``count`` 64-bit words of stream ``(seed, operand, draw)``; word ``i``
    is ``mix(key + (i + 1) * golden)``."""
    key = _stream_key(seed, operand, draw)
    with np.errstate(over="ignore"):
        ctr = key + (np.arange(1, count + 1, dtype=np.uint64) * _GOLDEN)
        return _mix(ctr)


def uniform01(seed: int, operand: int, draw: int, count: int, bits: int = 53) -> np.ndarray:
    """Uniform float64 on ``[0, 1)`` on a ``2**-bits`` grid (exact)."""
    w = random_u64(seed, operand, draw, count) >> np.uint64(64 - bits)
    return w.astype(np.float64) * (2.0 ** -bits)


def uniform_int(seed: int, operand: int, draw: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Uniform integers in ``{lo..hi}`` (multiply-shift reduction of 32 bits)."""
    span = hi - lo + 1
    w = random_u64(seed, operand, draw, count) >> np.uint64(32)
    return (lo + ((w * np.uint64(span)) >> np.uint64(32)).astype(np.int64)).astype(np.int64)


def gen_matrix(fmt: str, rows: int, cols: int, *, E: int = 8, seed: int = 0, operand: str = "A",
               spread: str = "uniform") -> np.ndarray:
    """Synthetic multi-component matrix, shape ``(c, cols, rows)`` (see module doc).

    ``spread='uniform'`` uses the integer exponent ``e ~ U{0..E}``;
    ``spread='eq1'`` uses the paper's ``(ru - 0.5) * exp(rn)`` leading part.
    """
    c, dt = FORMATS[fmt]
    op = _OPERANDS[operand] if isinstance(operand, str) else int(operand)
    count = rows * cols
    single = dt == np.float32
    if spread == "uniform":
        u = 2.0 * uniform01(seed, op, 0, count, bits=24 if single else 53) - 1.0
        e = uniform_int(seed, op, 1, count, 0, E)
        x0 = np.ldexp(u, e)
    elif spread == "eq1":
        ru = uniform01(seed, op, 0, count)
        u1 = uniform01(seed, op, 1, count)
        u2 = uniform01(seed, op, 2, count)
        rn = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        x0 = (ru - 0.5) * np.exp(rn)
    else:
        raise ValueError(f"unknown spread {spread!r}")
    out = np.empty((c, count), dtype=dt)
    out[0] = x0.astype(dt)
    scale = dt(2.0 ** (-24 if single else -53))
    for r in range(1, c):
        v = (uniform01(seed, op, 8 + r, count) - 0.5).astype(dt)
        out[r] = (out[r - 1] * scale) * v
    return out.reshape(c, cols, rows)


def gen_ds(rows: int, cols: int, *, E: int = 8, seed: int = 0, operand: str = "A", spread: str = "uniform"):
    """D+S matrix (a binary64 leading part and a binary32 trailing part):
    ``(hi, lo)`` of shapes ``(1, cols, rows)`` float64 and float32, hi drawn as
    the DD generator's leading component and ``lo = RN_f32(hi * 2**-53 * v)``
    with ``v`` uniform on ``[-0.5, 0.5)`` (so ``|lo| <= ulp(hi) / 2``)."""
    X = gen_matrix("dd", rows, cols, E=E, seed=seed, operand=operand, spread=spread)
    hi = np.ascontiguousarray(X[:1])
    return hi, X[1:2].astype(np.float32)


def gen_pair(fmt: str, m: int, n: int, k: int, *, E: int = 8, seed: int = 0, spread: str = "uniform"):
    """Operands of ``C = A B``: A is m x k as ``(c, k, m)``, B is k x n as ``(c, n, k)``."""
    A = gen_matrix(fmt, m, k, E=E, seed=seed, operand="A", spread=spread)
    B = gen_matrix(fmt, k, n, E=E, seed=seed, operand="B", spread=spread)
    return A, B


def log_uniform_sizes(seed: int, count: int, lo: int, hi: int, draw: int = 0) -> np.ndarray:
    """``round(lo * (hi/lo)**U)`` for a seeded uniform ``U`` (batched and served size mixes)."""
    U = uniform01(seed, 3, 40 + draw, count)
    return np.rint(lo * (hi / lo) ** U).astype(np.int64)
