"""Pins of the oracle's polynomial and integer products (CPU only)."""
import random

import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs

PRIMES = [998244353, 2013265921, 469762049, 167772161]
P62 = nt.largest_prime_below(62, 32)


def _py_conv(a, b, p):
    c = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[i + j] += int(x) * int(y)
    return [v % p for v in c]


@pytest.mark.parametrize("p", PRIMES + [P62])
@pytest.mark.parametrize("la,lb", [(1, 1), (1, 7), (5, 3), (16, 16), (33, 20)])
def test_schoolbook_matches_python(p, la, lb):
    r = random.Random(la * 100 + lb)
    a = [r.randrange(p) for _ in range(la)]
    b = [r.randrange(p) for _ in range(lb)]
    assert [int(x) for x in oracle.polymul_schoolbook(a, b, p)] == _py_conv(a, b, p)


@pytest.mark.parametrize("p", PRIMES + [P62])
@pytest.mark.parametrize("la,lb", [(1, 1), (3, 1), (100, 28), (512, 512), (1000, 3)])
def test_ntt_product_equals_schoolbook(p, la, lb):
    a = inputs.residues(p, la, inputs.CFG_TEST, la, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, lb, 1)
    assert np.array_equal(oracle.polymul_ntt(a, b, p), oracle.polymul_schoolbook(a, b, p))


def test_polymul_8k_random_point_evaluation():
    p, a, b = inputs.polymul_8k_inputs()
    c = oracle.polymul_schoolbook(a, b, p)
    assert c.size == 8191
    r = random.Random(3)
    for _ in range(8):
        x = r.randrange(p)
        assert oracle.horner(c, p, x) == oracle.horner(a, p, x) * oracle.horner(b, p, x) % p
    assert np.array_equal(oracle.polymul_ntt(a, b, p, 3), c)


def test_convolution_theorem():
    p = 469762049
    n = 512
    w = nt.root_of_unity(p, n, 3)
    a = inputs.residues(p, n // 2, inputs.CFG_TEST, 1)
    b = inputs.residues(p, n // 2, inputs.CFG_TEST, 2)
    c = oracle.polymul_schoolbook(a, b, p)
    pad = lambda v: np.concatenate([v.astype(np.uint64), np.zeros(n - v.size, dtype=np.uint64)])
    lhs = oracle.ntt(pad(c), p, w)
    rhs = np.array([oracle.mulmod(int(x), int(y), p) for x, y in zip(oracle.ntt(pad(a), p, w), oracle.ntt(pad(b), p, w))], dtype=np.uint64)
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("na,nb", [(1, 1), (2, 1), (3, 3), (10, 7), (64, 64), (101, 50)])
def test_intmul_schoolbook_and_3prime_match_python_int(na, nb):
    a = inputs.limbs16(na, inputs.CFG_TEST, na, 0)
    b = inputs.limbs16(nb, inputs.CFG_TEST, nb, 1)
    ref = oracle.intmul_pyint(a, b)
    assert ref.size == (na + nb + 1) // 2
    assert np.array_equal(oracle.intmul_schoolbook(a, b), ref)
    assert np.array_equal(oracle.intmul_3prime(a, b), ref)


def test_intmul_3prime_medium_and_closed_form():
    a, b = inputs.intmul_inputs(1 << 12, inputs.CFG_TEST, 5)
    assert np.array_equal(oracle.intmul_3prime(a, b), oracle.intmul_pyint(a, b))
    # (2^(16n) - 1)^2 = 2^(32n) - 2^(16n+1) + 1
    n = 1000
    ff = np.full(n, 0xFFFF, dtype=np.uint16)
    c = oracle.intmul_3prime(ff, ff)
    v = int.from_bytes(c.astype("<u4").tobytes(), "little")
    assert v == (1 << (32 * n)) - (1 << (16 * n + 1)) + 1


def test_garner_third_digit_vanishes():
    # coefficients of the product are < n (2^16-1)^2 < 2^53 < p1 p2: x3 = 0
    a, b = inputs.intmul_inputs(1 << 10, inputs.CFG_TEST, 6)
    r = [oracle.polymul_ntt(a.astype(np.uint64), b.astype(np.uint64), q) for q in oracle.INTMUL_PRIMES]
    x1, x2, x3 = oracle.garner_digits(*r)
    assert np.all(x3 == 0)
    exact = oracle.polymul_schoolbook(a.astype(np.uint64), b.astype(np.uint64), (1 << 61) - 1)
    value = x1.astype(object) + oracle.INTMUL_PRIMES[0] * x2.astype(object)
    assert all(int(v) == int(e) for v, e in zip(value, exact))


def test_limb_residues():
    a, b = inputs.intmul_inputs(300, inputs.CFG_TEST, 7)
    c = oracle.intmul_schoolbook(a, b)
    q = (1 << 61) - 1
    assert oracle.limbs32_mod(c, q) == oracle.limbs16_mod(a, q) * oracle.limbs16_mod(b, q) % q
