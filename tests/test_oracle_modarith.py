"""Exhaustive pins of the word-generic forms of Functions 2, 6, 8 and 13 (section 2)
at n = 8: every modulus the function admits and every pair of residues, against the
definition (x + y) rem p / (x y) rem p, with each proposition's stated bound."""
import pytest

from oracle import modarith as ma
from oracle import numtheory as nt

N = 8


def test_function2_add_min_exhaustive():
    # m <= n - 1: every p < 2^(n-1) (p = 0 would mean "mod 2^n" and is excluded)
    for p in range(1, 1 << (N - 1)):
        for x in range(p):
            for y in range(p):
                assert ma.add_mod_min(x, y, p, N) == (x + y) % p
                assert ma.sub_mod_min(x, y, p, N) == (x - y) % p


def test_function6_barrett_exhaustive_with_prop1_bound():
    for p in range(2, 1 << N):
        prm = nt.barrett_params(p, N)
        bound = prm["alpha"] * p
        step = max(1, bound // 4096)
        for a in list(range(0, bound, step)) + [bound - 1]:
            d, corrections = ma.reduce_barrett(a, p, N)
            assert d == a % p
            assert corrections <= prm["h"]


def test_function8_fixed_multiplicand_exhaustive_prop4():
    for p in range(2, 1 << N):
        for y in range(p):
            psi = nt.shoup_constant(y, p, N)
            for x in range(p):
                r, d = ma.mul_mod_shoup(x, y, psi, p, N)
                assert r == x * y % p
                assert 0 <= d < 2 * p


def test_function13_montgomery_exhaustive_prop7():
    for m in (N - 1, N):
        for p in range(3, 1 << m, 2):
            rho, _ = nt.montgomery_constants(p, m)
            for x in range(p):
                for y in range(p):
                    a = x * y
                    r, d = ma.reduce_montgomery(a, p, m, N)
                    assert r == a * rho % p
                    assert d < 2 * p


def test_montgomery_representation_product():
    # section 2.3: Function 13 applied to x~ y~ gives the representation of x y
    p, m, n = 251, 8, 8
    for x in range(0, p, 7):
        for y in range(0, p, 5):
            xt, yt = (x << m) % p, (y << m) % p
            r, _ = ma.reduce_montgomery(xt * yt, p, m, n)
            assert r == ((x * y) << m) % p


@pytest.mark.parametrize("p", [998244353, 2013265921, 469762049, 167772161])
def test_word32_forms_random(p):
    import random
    rnd = random.Random(p)
    n = 32
    for _ in range(2000):
        x, y = rnd.randrange(p), rnd.randrange(p)
        psi = nt.shoup_constant(y, p, n)
        assert ma.mul_mod_shoup(x, y, psi, p, n)[0] == x * y % p
        assert ma.reduce_barrett(x * y, p, n)[0] == x * y % p
        rho, _ = nt.montgomery_constants(p, 32)
        assert ma.reduce_montgomery(x * y, p, 32, n)[0] == x * y * rho % p
        assert ma.add_mod_min(x, y, p, n) == (x + y) % p
