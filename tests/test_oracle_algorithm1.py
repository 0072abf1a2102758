"""Proposition 15 (section 5.1): Algorithm 1 returns A(w^[i]_k), i < lambda n1 --
checked against the TFT definition and against the C oracle's transform."""
import random

import numpy as np
import pytest

import oracle
from oracle import algorithm1 as alg
from oracle import numtheory as nt


@pytest.mark.parametrize("p,g", [(998244353, 3), (2013265921, 31), (469762049, 3)])
@pytest.mark.parametrize("k,k1", [(1, 0), (2, 1), (4, 2), (5, 2), (6, 3), (6, 6), (7, 1)])
def test_algorithm1_full_length_matches_tft(p, g, k, k1):
    n, n1 = 1 << k, 1 << k1
    w = nt.root_of_unity(p, n, g)
    r = random.Random(k * 10 + k1)
    a = [r.randrange(p) for _ in range(n)]
    out = alg.algorithm1(a, n, n, n1, w, p)
    assert out == alg.tft_definition(a, n, n, w, p)
    nat = oracle.ntt(np.array(a, dtype=np.uint64), p, w)
    assert out == [int(x) for x in oracle.tft_order(nat)]


@pytest.mark.parametrize("k,k1,l", [(5, 2, 17), (5, 2, 20), (6, 3, 9), (6, 1, 33), (4, 2, 4)])
def test_algorithm1_truncated(k, k1, l):
    p, g = 469762049, 3
    n, n1 = 1 << k, 1 << k1
    w = nt.root_of_unity(p, n, g)
    r = random.Random(l)
    a = [r.randrange(p) for _ in range(l)]
    lam = -(-l // n1)
    out = alg.algorithm1(a, l, n, n1, w, p)
    assert len(out) == lam * n1
    assert out == alg.tft_definition(a, lam * n1, n, w, p)


def test_mirror_definition():
    # [i]_k reverses the binary expansion i_0 + 2 i_1 + ... of i in length k
    assert alg.mirror(1, 3) == 4 and alg.mirror(6, 3) == 3 and alg.mirror(0, 5) == 0
    for k in range(1, 9):
        for i in range(1 << k):
            assert alg.mirror(alg.mirror(i, k), k) == i
            assert alg.mirror(i, k) == oracle.bitrev(i, k)


@pytest.mark.parametrize("k,l", [(0, 1), (1, 1), (3, 5), (4, 1), (4, 9), (5, 17), (5, 32), (6, 40), (6, 63)])
def test_itft_definition_inverts_the_tft(k, l):
    # the inverse TFT by its definition (a linear solve) recovers the l-tuple from its l values
    p, g = 998244353, 3
    n = 1 << k
    w = nt.root_of_unity(p, n, g)
    r = random.Random(100 * k + l)
    a = [r.randrange(p) for _ in range(l)]
    v = alg.tft_definition(a, l, n, w, p)
    assert alg.itft_definition(v, l, n, w, p) == a


def test_itft_definition_full_length_is_the_inverse_transform():
    # with l = n the inverse TFT is the inverse transform of the values put back in natural order
    p, g, k = 469762049, 3, 5
    n = 1 << k
    w = nt.root_of_unity(p, n, g)
    r = random.Random(7)
    vals = [r.randrange(p) for _ in range(n)]
    nat = np.zeros(n, dtype=np.uint64)
    for i in range(n):
        nat[alg.mirror(i, k)] = vals[i]
    assert alg.itft_definition(vals, n, n, w, p) == [int(x) for x in oracle.intt(nat, p, w)]


@pytest.mark.parametrize("k,lin,lout", [(4, 16, 16), (5, 7, 20), (6, 33, 5), (6, 1, 64)])
def test_tft_helper_matches_definition(k, lin, lout):
    p, g = 2013265921, 31
    n = 1 << k
    w = nt.root_of_unity(p, n, g)
    r = random.Random(lin * 7 + lout)
    a = [r.randrange(p) for _ in range(lin)]
    assert [int(x) for x in oracle.tft(np.array(a, dtype=np.uint64), n, lout, p, w)] == alg.tft_definition(a, lout, n, w, p)
