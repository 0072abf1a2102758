"""Pins of the oracle's number theory (CPU only).

The oracle's primality test, generators and constants are checked against sympy's
independent routines, the moduli the paper prints, and the defining identities.
"""
import os
import random

import pytest
import sympy

from oracle import numtheory as nt

HERE = os.path.dirname(os.path.abspath(__file__))
CONFIG_PRIMES = [(998244353, 3), (2013265921, 31), (469762049, 3), (167772161, 3)]


def _paper_primes():
    rows = []
    with open(os.path.join(HERE, "golden", "paper_primes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p, k, l = line.split()[:3]
                rows.append((int(p), int(k), int(l)))
    return rows


@pytest.mark.parametrize("p,k,l", _paper_primes())
def test_paper_moduli_are_primes_of_fft_form(p, k, l):
    # Section 1: fields F_p with p = k 2^l + 1 and l large.
    assert nt.is_prime(p) and sympy.isprime(p)
    assert p == k * (1 << l) + 1 and k % 2 == 1
    assert nt.two_adic(p) == (k, l)


def test_is_prime_matches_sympy_small_exhaustive():
    for n in range(0, 20000):
        assert nt.is_prime(n) == sympy.isprime(n), n


def test_is_prime_matches_sympy_random_64bit():
    r = random.Random(1)
    for _ in range(3000):
        n = r.getrandbits(64) | 1
        assert nt.is_prime(n) == sympy.isprime(n), n
    # strong pseudoprimes to several small bases must be rejected
    for n in (3215031751, 2152302898747, 3474749660383, 341550071728321, 3825123056546413051):
        assert not nt.is_prime(n)


@pytest.mark.parametrize("p,g", CONFIG_PRIMES)
def test_config_generators_are_primitive(p, g):
    assert nt.is_generator(g, p)
    assert sympy.is_primitive_root(g, p)
    assert nt.smallest_generator(p) == sympy.primitive_root(p)


@pytest.mark.parametrize("p,g", CONFIG_PRIMES)
def test_roots_have_exact_power_of_two_order(p, g):
    k, l = nt.two_adic(p)
    for log2n in range(0, l + 1):
        n = 1 << log2n
        w = nt.root_of_unity(p, n, g)
        assert pow(w, n, p) == 1
        if n > 1:
            assert pow(w, n // 2, p) == p - 1
        assert sympy.n_order(w, p) == n
    with pytest.raises(ValueError):
        nt.root_of_unity(p, 1 << (l + 1), g)


def test_sixty_two_bit_prime_rule():
    p = nt.largest_prime_below(62, 32)
    assert p < (1 << 62) and p % (1 << 32) == 1
    assert sympy.isprime(p) and nt.is_prime(p)
    k = (p - 1) >> 32
    # no larger candidate k 2^32 + 1 below 2^62 is prime
    for kk in range(k + 1, ((1 << 62) - 2 >> 32) + 1):
        assert not sympy.isprime((kk << 32) + 1)
    assert 4 * p < (1 << 64)
    g = nt.smallest_generator(p)
    assert g == sympy.primitive_root(p)
    w = nt.root_of_unity(p, 1 << 21, g)
    assert sympy.n_order(w, p) == 1 << 21


# Montgomery's representation needs p < 2^m: only those pairs
@pytest.mark.parametrize("p,m", [(p, m) for p in (998244353, 2013265921, 469762049, 167772161, 97, 257, 65537)
                                 for m in (8, 16, 32) if p < (1 << m)])
def test_montgomery_constants_identity(p, m):
    rho, chi = nt.montgomery_constants(p, m)
    assert rho * (1 << m) - chi * p == 1
    assert 0 < chi < (1 << m) and 0 < rho < p


@pytest.mark.parametrize("p", [998244353, 2013265921, 469762049, 167772161])
def test_barrett_and_shoup_constants(p):
    n = 32
    prm = nt.barrett_params(p, n)
    assert (1 << (prm["r"] - 1)) < p <= (1 << prm["r"])
    assert prm["t"] >= prm["r"] and prm["s"] + prm["t"] <= n + prm["r"] - 1
    assert prm["q"] < (1 << n)
    # Table 3 column by bit size: 30-bit primes -> h = 1, the 31-bit prime -> h = 2
    assert prm["h"] == (1 if prm["r"] <= n - 2 else 2)
    for y in (0, 1, 2, p // 2, p - 1):
        psi = nt.shoup_constant(y, p, n)
        assert psi < (1 << n)
        assert psi * p <= (y << n) < (psi + 1) * p
