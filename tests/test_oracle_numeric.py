"""Pins of the oracle's FP64 modular product (section 3.3, Function 16) against the
integer definition (a1 a2) mod p, and of Proposition 13's range of the uncorrected
value, for primes up to the bound 2^50 and operands in the ranges the transforms
feed it (canonical, below 2p, below 4p)."""
import numpy as np
import pytest

from oracle import numeric, numtheory


def _prime_below(bits, l):
    return numtheory.largest_prime_below(bits, l)


def _primes():
    out = [998244353, _prime_below(40, 20), _prime_below(48, 20), _prime_below(49, 20), 63 * 2 ** 44 + 1]
    assert numtheory.is_prime(63 * 2 ** 44 + 1)
    return out


def _check(p, a1, a2):
    r, e = numeric.mul_mod_fma(a1, a2, p)
    assert r == a1 * a2 % p, (p, a1, a2, r)
    assert -p <= e < 2 * p, (p, a1, a2, e)


@pytest.mark.parametrize("p", _primes())
def test_function16_canonical_operands(p):
    assert p < 2 ** 50
    g = np.random.default_rng(p % 1000003)
    edge = [0, 1, 2, p - 1, p - 2, p // 2, (p + 1) // 2, int(np.sqrt(p))]
    for a1 in edge:
        for a2 in edge:
            _check(p, a1, a2)
    for _ in range(3000):
        _check(p, int(g.integers(0, p)), int(g.integers(0, p)))


@pytest.mark.parametrize("bits,bound", [(48, 4), (49, 2)])
def test_function16_lazy_operand_ranges(bits, bound):
    """The transforms multiply an operand below 4p (p < 2^48) or 2p (p < 2^49) by a
    canonical twiddle: a1 a2 < 2^50 p still holds."""
    p = _prime_below(bits, 20)
    assert bound * p * p < 2 ** 50 * p
    g = np.random.default_rng(bits)
    for a1 in [bound * p - 1, bound * p - 2, p, p + 1]:
        for a2 in [p - 1, 1, p // 3]:
            _check(p, a1, a2)
    for _ in range(3000):
        _check(p, int(g.integers(0, bound * p)), int(g.integers(0, p)))


def test_fma_emulation_is_exact_rounding():
    # x y + z with x y not representable: the FMA keeps the low bits a plain product loses
    x = float(2 ** 52 + 1)
    h = x * x
    assert numeric.fma(x, x, -h) == float((2 ** 52 + 1) ** 2 - int(h))
    assert numeric.fma(3.0, 5.0, 1.0) == 16.0
