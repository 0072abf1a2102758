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
