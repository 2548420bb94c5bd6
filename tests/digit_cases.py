"""Inputs on and next to the rounding boundaries of the INT8 digits (test
helper, no arithmetic of the method): values built from exact rationals and
written as normalized binary64 expansions."""
from fractions import Fraction

import numpy as np


def greedy_expansion(v: Fraction, c: int):
    """v as c binary64 components, each the nearest double to what the earlier
    ones leave (a normalized expansion; exact when v fits)."""
    out = []
    for _ in range(c):
        out.append(float(v))
        v -= Fraction(out[-1])
    return out


def tie_cases(c: int, D: int, E: int, seed: int):
    """Values on or next to a rounding boundary of some digit: exact ties
    (half a unit of digit s, after random digits above it), ties moved by a
    tiny amount either way (the move held in a lower component), negatives."""
    rng = np.random.default_rng(seed)
    cases = []
    top = min(D, (53 * c - 20) // 7)  # digits whose boundary the expansion can carry exactly
    for s in list(range(1, min(top, 6) + 1)) + list(rng.integers(1, top + 1, 6)):
        s = int(s)
        head = sum((Fraction(int(rng.integers(-64, 65))) * Fraction(2) ** (E - 6 - 7 * (t - 1)) for t in range(2, s)),
                   Fraction(int(rng.integers(-31, 32))) * Fraction(2) ** (E - 6))
        u = Fraction(2) ** (E - 6 - 7 * (s - 1))
        for tiny in (Fraction(0), u * Fraction(2) ** -70, -u * Fraction(2) ** -70):
            for sign in (1, -1):
                v = sign * (head + u / 2 + tiny)
                if abs(v) < Fraction(2) ** (E - 1) or abs(v) >= Fraction(2) ** E:
                    v = sign * (Fraction(2) ** (E - 1) + u / 2 + tiny)  # keep the row's E
                cases.append(greedy_expansion(v, c))
    return cases
