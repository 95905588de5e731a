"""Exact float32 arithmetic for brute-force pins: every operation is evaluated on exact rationals and
rounded once to the nearest float32 (ties to even), the IEEE-754 definition of a correctly rounded
binary32 operation. Slow, for a handful of values only."""
from fractions import Fraction

import numpy as np

F32 = np.float32


def rnd(x: Fraction) -> F32:
    """Nearest float32 to the exact rational x (ties to even)."""
    f = F32(float(x))                   # may be off by one ulp through double rounding
    best, bestd = None, None
    for c in (np.nextafter(f, F32(-np.inf)), f, np.nextafter(f, F32(np.inf))):
        if not np.isfinite(c):
            continue
        d = abs(Fraction(float(c)) - x)
        if bestd is None or d < bestd or (d == bestd and (int(c.view(np.uint32)) & 1) == 0):
            best, bestd = c, d
    return F32(best)


def Fr(a) -> Fraction:
    return Fraction(float(F32(a)))


def add(a, b):
    return rnd(Fr(a) + Fr(b))


def sub(a, b):
    return rnd(Fr(a) - Fr(b))


def mul(a, b):
    return rnd(Fr(a) * Fr(b))


def fma(a, b, c):
    return rnd(Fr(a) * Fr(b) + Fr(c))


def div(a, b):
    return rnd(Fr(a) / Fr(b))
