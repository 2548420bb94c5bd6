"""Pins of the oracle's error-free transformations and renormalization against
exact rational arithmetic (not against themselves)."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle.exact as X

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _cases(seed=0, n=3000):
    rnd = random.Random(seed)
    out = []
    for _ in range(n):
        a = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60)
        b = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60)
        out.append((a, b))
    # adversarial: ties, exact cancellation, huge gaps, signed zeros, equal magnitudes
    out += [(1.0, 2.0 ** -53), (1.0 + 2.0 ** -52, 2.0 ** -53), (1.0, -1.0), (0.0, -0.0), (-0.0, -0.0),
            (2.0 ** 60, 2.0 ** -60), (3.0, -3.0 * (1 - 2.0 ** -53)), (2.0 ** -1000, 2.0 ** 900),
            (1.5, 1.5), (-(2.0 ** 52), 0.5), (2.0 ** 53, 1.0)]
    return out


def test_two_sum_exact(orc):
    for a, b in _cases():
        s, e = orc.two_sum(a, b)
        assert s == a + b  # s is the rounded sum
        assert Fraction(s) + Fraction(e) == Fraction(a) + Fraction(b)
        assert abs(e) <= math.ulp(s) / 2 or s == 0


def test_two_sum_f32_exact(orc):
    for a, b in _cases(1, 1000):
        a32, b32 = np.float32(a), np.float32(b)
        if not (np.isfinite(a32) and np.isfinite(b32)):
            continue
        s, e = orc.two_sum_f(a32, b32)
        assert s == np.float32(a32 + b32)
        assert Fraction(float(s)) + Fraction(float(e)) == Fraction(float(a32)) + Fraction(float(b32))


def test_two_prod_exact(orc):
    for a, b in _cases(2, 2000):
        p, e = orc.two_prod(a, b)
        if p == 0 or abs(p) < 2.0 ** -900:
            continue  # below the underflow limit of the error term
        assert Fraction(p) + Fraction(e) == Fraction(a) * Fraction(b)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_renorm_preserves_sum_and_matches_written_spec(orc, n):
    rnd = random.Random(n)
    for trial in range(400):
        x = [rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-70, 10) for _ in range(n)]
        if trial % 5 == 0:  # overlapping, cancelling terms
            x[1] = -x[0] + rnd.uniform(-1, 1) * 2.0 ** -40
        y = orc.renorm(x)
        assert X.value(y) == X.value(x)
        # an independent Python implementation of the same written procedure
        assert list(y) == X.renorm_py(x)
        # the leading term is nonzero iff the sum is
        assert (y[0] != 0) == (X.value(x) != 0)


def test_renorm_leading_term_near_value(orc):
    """For well-separated inputs the leading term is the sum rounded to nearest."""
    rnd = random.Random(7)
    for _ in range(500):
        x0 = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-30, 30)
        x = [x0, x0 * 2.0 ** -60 * rnd.uniform(-1, 1), x0 * 2.0 ** -120 * rnd.uniform(-1, 1)]
        y = orc.renorm(x)
        assert y[0] == float(X.value(x))  # float(Fraction) rounds correctly


def test_renorm_f32(orc):
    rnd = random.Random(3)
    for _ in range(300):
        x = np.array([rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-30, 10) for _ in range(3)], dtype=np.float32)
        y = orc.renorm(x)
        assert X.value(y) == X.value(x)
        assert [float(v) for v in y] == [float(v) for v in X.renorm_py(x, f32=True)]


def test_exact_sum_is_correctly_rounded_greedy_expansion(orc):
    rnd = random.Random(11)
    for _ in range(300):
        vals = [rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-200, 50) for _ in range(rnd.randint(1, 12))]
        exact = sum((Fraction(v) for v in vals), Fraction(0))
        out = orc.exact_sum(vals, 4)
        rest = exact
        for r in range(4):
            assert out[r] == float(rest)  # greedy: each term is the remainder rounded to nearest
            rest -= Fraction(out[r])
