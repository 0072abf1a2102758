"""Pins of the oracle's transforms (CPU only): the C definitions against Python-integer
re-derivations, closed forms of the transform, the inverse, and Horner evaluation."""
import random

import numpy as np
import pytest

import oracle
from oracle import numtheory as nt

PRIMES = [(998244353, 3), (2013265921, 31), (469762049, 3), (167772161, 3)]
P62 = nt.largest_prime_below(62, 32)


def _py_dft(a, p, w):
    n = len(a)
    return [sum(int(a[j]) * pow(w, i * j, p) for j in range(n)) % p for i in range(n)]


def _rand(p, n, seed):
    r = random.Random(seed)
    return np.array([r.randrange(p) for _ in range(n)], dtype=np.uint64)


@pytest.mark.parametrize("p,g", PRIMES + [(P62, None)])
def test_mulmod_against_python_ints(p, g):
    r = random.Random(p)
    vals = [0, 1, 2, p - 1, p - 2, p // 2] + [r.randrange(p) for _ in range(300)]
    for x in vals:
        for y in vals[:20]:
            assert oracle.mulmod(x, y, p) == x * y % p
    assert oracle.powmod(3, p - 1, p) == 1
    for x in vals[1:40]:
        assert oracle.mulmod(x, oracle.invmod(x, p), p) == 1


@pytest.mark.parametrize("p,g", PRIMES + [(P62, None)])
@pytest.mark.parametrize("log2n", [0, 1, 2, 3, 5, 6])
def test_dft_definition_matches_python(p, g, log2n):
    n = 1 << log2n
    w = nt.root_of_unity(p, n, g)
    a = _rand(p, n, log2n)
    assert [int(x) for x in oracle.dft(a, p, w)] == _py_dft(a, p, w)


@pytest.mark.parametrize("p,g", PRIMES + [(P62, None)])
@pytest.mark.parametrize("log2n", [1, 2, 4, 7, 10])
def test_textbook_ntt_equals_definition(p, g, log2n):
    n = 1 << log2n
    w = nt.root_of_unity(p, n, g)
    a = _rand(p, n, 100 + log2n)
    assert np.array_equal(oracle.ntt(a, p, w), oracle.dft(a, p, w))
    assert np.array_equal(oracle.intt(oracle.ntt(a, p, w), p, w), a)


@pytest.mark.parametrize("p,g", PRIMES)
def test_closed_forms(p, g):
    n = 256
    w = nt.root_of_unity(p, n, g)
    delta0 = np.zeros(n, dtype=np.uint64)
    delta0[0] = 1
    assert np.all(oracle.ntt(delta0, p, w) == 1)                      # FFT(delta_0) = (1,...,1)
    out = oracle.ntt(np.ones(n, dtype=np.uint64), p, w)               # FFT(1,...,1) = n delta_0
    assert out[0] == n % p and np.all(out[1:] == 0)
    for j in (1, 3, 77, 255):
        dj = np.zeros(n, dtype=np.uint64)
        dj[j] = 1
        out = oracle.ntt(dj, p, w)                                     # FFT(delta_j)_i = w^(ij)
        assert all(int(out[i]) == pow(w, i * j, p) for i in range(n))
    a, b = _rand(p, n, 5), _rand(p, n, 6)                              # linearity
    lhs = oracle.ntt((a + 7 * b) % p, p, w)
    rhs = (oracle.ntt(a, p, w) + 7 * oracle.ntt(b, p, w)) % p
    assert np.array_equal(lhs, rhs)
    pm1 = np.full(n, p - 1, dtype=np.uint64)                           # FFT(-1,...,-1) = -n delta_0
    out = oracle.ntt(pm1, p, w)
    assert out[0] == (-n) % p and np.all(out[1:] == 0)


@pytest.mark.parametrize("p,g", PRIMES)
def test_horner_is_transform_entry(p, g):
    n = 1024
    w = nt.root_of_unity(p, n, g)
    a = _rand(p, n, 9)
    full = oracle.ntt(a, p, w)
    idx = [0, 1, 2, 511, 512, 1023, 333]
    xs = [pow(w, i, p) for i in idx]
    assert [int(v) for v in oracle.horner_many(a, p, xs)] == [int(full[i]) for i in idx]
    assert oracle.horner(a, p, 1) == int(a.astype(object).sum() % p)


def test_tft_order_is_mirror_permutation():
    p, g = 998244353, 3
    k = 6
    n = 1 << k
    w = nt.root_of_unity(p, n, g)
    a = _rand(p, n, 11)
    nat = oracle.ntt(a, p, w)
    tft = oracle.tft_order(nat)
    for i in range(n):
        assert tft[i] == nat[oracle.bitrev(i, k)]
        assert int(tft[i]) == oracle.horner(a, p, pow(w, oracle.bitrev(i, k), p))
