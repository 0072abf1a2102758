"""Word-size-generic forms of the paper's integer modular primitives (section 2).

Test infrastructure only.  Each function emulates n-bit unsigned words (U) and
2n-bit words (L) with explicit wrap-around, follows the steps of the named Function
in the paper's order, and returns the value together with the internal quantity its
proposition bounds, so that the tests can check the propositions exhaustively for
small n (every p < 2^n, every pair of residues) against the plain definition.
"""
from __future__ import annotations

from .numtheory import barrett_params, montgomery_constants


def _wrap(x: int, bits: int) -> int:
    return x & ((1 << bits) - 1)


def add_mod_min(x: int, y: int, p: int, n: int) -> int:
    """Function 2: a = x + y in U, then min(a, a - p) in U; needs p < 2^(n-1)."""
    a = _wrap(x + y, n)
    return min(a, _wrap(a - p, n))


def sub_mod_min(x: int, y: int, p: int, n: int) -> int:
    """Subtraction 'in a similar manner' (section 2.1.1): a = x - y in U, then
    min(a, a + p) in U."""
    a = _wrap(x - y, n)
    return min(a, _wrap(a + p, n))


def reduce_barrett(a: int, p: int, n: int) -> tuple[int, int]:
    """Function 6 with Table 3's parameters: b = a >> s, c = (b q) >> t, d = a - c p,
    then subtract p while d >= p.  Returns (d, number of corrections); Proposition 1
    bounds the corrections by h for a < alpha p."""
    prm = barrett_params(p, n)
    L = 2 * n
    b = a >> prm["s"]
    c = _wrap(b * prm["q"], L) >> prm["t"]
    d = _wrap(a - c * p, L)
    steps = 0
    while d >= p:
        d -= p
        steps += 1
    return d, steps


def mul_mod_shoup(x: int, y: int, psi: int, p: int, n: int) -> tuple[int, int]:
    """Function 8 (fixed multiplicand y, psi = floor(2^n y / p)):
    c = (x psi) >> n; d = x y - c p in L; return d - p if d >= p else d.
    Returns (result, d before the last line); Proposition 4's proof gives d < 2p."""
    L = 2 * n
    c = _wrap(x * psi, L) >> n
    d = _wrap(x * y - c * p, L)
    return (d - p if d >= p else d), d


def reduce_montgomery(a: int, p: int, m: int, n: int) -> tuple[int, int]:
    """Function 13: b = (a chi) & (2^m - 1); c = a + b p in L; d = c >> m;
    if c < a (overflow) return d - p; return d - p if d >= p else d.
    Returns ((a rho) rem p, d); Proposition 7 gives d < 2p."""
    rho, chi = montgomery_constants(p, m)
    L = 2 * n
    mu = (1 << m) - 1
    b = _wrap(a * chi, n) & mu
    c = _wrap(a + b * p, L)
    d = c >> m
    if c < a:
        return _wrap(d - p, n), d
    return (d - p if d >= p else d), d
