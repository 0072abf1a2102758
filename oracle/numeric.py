"""Modular products over a numeric type (section 3 of the paper), for pinning the
FP64 arithmetic.

Test infrastructure only.  Python floats are IEEE-754 binary64 numbers (52 explicit
mantissa bits) with round-to-nearest, the setting of section 3.  The fused
multiply-add is emulated exactly: the exact value x y + z is formed as a rational
number and rounded once to the nearest double (the division of two integers in
Python is correctly rounded).
"""
from __future__ import annotations

import math
from fractions import Fraction


def fma(x: float, y: float, z: float) -> float:
    """x y + z rounded once to the nearest double (IEEE 754-2008 fusedMultiplyAdd)."""
    return float(Fraction(x) * Fraction(y) + Fraction(z))


def mul_mod_fma(a1: int, a2: int, p: int) -> tuple[int, int]:
    """Function 16 (section 3.3): (a1 a2) rem p for a1 a2 < 2^50 p, with u = 1/p
    rounded to nearest.  Returns (result, e) where e = d + l is the value before the
    two corrections (Proposition 13: e = a1 a2 - c p with c within one of
    floor(a1 a2 / p), so -p <= e < 2p)."""
    x, y, pf = float(a1), float(a2), float(p)
    u = 1.0 / pf
    h = x * y
    lo = fma(x, y, -h)
    b = h * u
    c = math.floor(b)
    d = fma(-float(c), pf, h)
    e = d + lo
    r = e
    if r >= pf:
        r -= pf
    if r < 0:
        r += pf
    return int(r), int(e)
