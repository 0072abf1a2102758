"""Pins of the oracle's polynomial matrix product (section 5.2) against facts that do
not go through its own formula: evaluation at random points (a ring morphism
F_p[x] -> F_p, so C(x) = A(x) B(x) as matrices over F_p), the degree-0 case (an
ordinary matrix product, numpy over Python integers), the 1 x 1 case (the
polynomial product), the transpose law (A B)^T = B^T A^T (F_p[x] is commutative),
the identity matrix, and the distributive law.  The integer matrix product of
section 5.3 is pinned by its images modulo random 61-bit q, a closed form and the
1 x 1 and identity cases."""
import numpy as np
import pytest

import oracle
from paper_1407_3383_amd import inputs

P = 469762049  # the prime of section 5.2's matrix product table


def _mat(n, d, item, stream, p=P):
    return inputs.residues(p, n * n * d, inputs.CFG_TEST, item, stream).reshape(n, n, d)


def _eval_py(poly, x, p):
    r = 0
    for c in reversed([int(v) for v in poly]):
        r = (r * x + c) % p
    return r


@pytest.mark.parametrize("n,d", [(1, 5), (2, 3), (3, 17), (5, 40)])
def test_evaluation_morphism(n, d):
    A, B = _mat(n, d, 9100 + n, 0), _mat(n, d, 9100 + n, 1)
    C = oracle.polymatmul(A, B, P)
    assert C.shape == (n, n, 2 * d - 1)
    g = np.random.default_rng(n * 1000 + d)
    for _ in range(4):
        x = int(g.integers(0, P))
        ea = [[_eval_py(A[i, l], x, P) for l in range(n)] for i in range(n)]
        eb = [[_eval_py(B[l, j], x, P) for j in range(n)] for l in range(n)]
        for i in range(n):
            for j in range(n):
                want = sum(ea[i][l] * eb[l][j] for l in range(n)) % P
                assert _eval_py(C[i, j], x, P) == want, (i, j, x)


def test_degree_zero_is_a_matrix_product():
    n = 7
    A, B = _mat(n, 1, 9200, 0), _mat(n, 1, 9200, 1)
    want = (A[:, :, 0].astype(object).dot(B[:, :, 0].astype(object))) % P
    got = oracle.polymatmul(A, B, P)[:, :, 0]
    assert (got.astype(object) == want).all()


def test_one_by_one_is_the_polynomial_product():
    A, B = _mat(1, 300, 9300, 0), _mat(1, 300, 9300, 1)
    np.testing.assert_array_equal(oracle.polymatmul(A, B, P)[0, 0], oracle.polymul_schoolbook(A[0, 0], B[0, 0], P))


def test_transpose_law():
    n, d = 4, 9
    A, B = _mat(n, d, 9400, 0), _mat(n, d, 9400, 1)
    lhs = oracle.polymatmul(A, B, P).transpose(1, 0, 2)
    rhs = oracle.polymatmul(np.ascontiguousarray(B.transpose(1, 0, 2)), np.ascontiguousarray(A.transpose(1, 0, 2)), P)
    np.testing.assert_array_equal(lhs, rhs)


def test_identity_matrix():
    n, d = 5, 6
    A = _mat(n, d, 9500, 0)
    eye = np.zeros((n, n, d), dtype=np.uint64)
    for i in range(n):
        eye[i, i, 0] = 1
    want = np.zeros((n, n, 2 * d - 1), dtype=np.uint64)
    want[:, :, :d] = A
    np.testing.assert_array_equal(oracle.polymatmul(A, eye, P), want)
    np.testing.assert_array_equal(oracle.polymatmul(eye, A, P), want)


def test_distributive_law():
    n, d = 3, 11
    A, B, D = _mat(n, d, 9600, 0), _mat(n, d, 9600, 1), _mat(n, d, 9600, 2)
    left = oracle.polymatmul(A, (B + D) % P, P)
    right = (oracle.polymatmul(A, B, P) + oracle.polymatmul(A, D, P)) % P
    np.testing.assert_array_equal(left, right)


def test_single_coefficient_matches_full_product_and_extremes():
    n, d = 4, 33
    A, B = _mat(n, d, 9700, 0), _mat(n, d, 9700, 1)
    C = oracle.polymatmul(A, B, P)
    for (i, j, k) in [(0, 0, 0), (3, 1, 2 * d - 2), (2, 3, d - 1), (1, 2, d)]:
        assert oracle.polymatmul_coeff(A, B, P, i, j, k) == int(C[i, j, k])
    # all coefficients p - 1: C_ij[k] = n * (number of (s, t), s + t = k) * (p - 1)^2
    full = np.full((n, n, d), P - 1, dtype=np.uint64)
    Cf = oracle.polymatmul(full, full, P)
    for k in (0, d - 1, 2 * d - 2):
        terms = min(k, 2 * d - 2 - k) + 1
        assert int(Cf[1, 2, k]) == n * terms * (P - 1) ** 2 % P


def test_64_bit_prime():
    p = 4611685941117976577
    n, d = 2, 5
    A, B = _mat(n, d, 9800, 0, p), _mat(n, d, 9800, 1, p)
    C = oracle.polymatmul(A, B, p)
    x = 123456789123
    for i in range(n):
        for j in range(n):
            want = sum(_eval_py(A[i, l], x, p) * _eval_py(B[l, j], x, p) for l in range(n)) % p
            assert _eval_py(C[i, j], x, p) == want


# ---------------------------------------------------------------- integer matrices

def _limbs(n, na, item, stream):
    return inputs.limbs32(n * n * na, inputs.CFG_TEST, item, stream).reshape(n, n, na)


def test_integer_matrix_product_modular_images():
    """C mod q = (A mod q)(B mod q) mod q for random 61-bit q (a ring morphism Z -> Z/q),
    the matrix product over Z/q taken by numpy over Python integers."""
    n, na = 3, 9
    A, B = _limbs(n, na, 9900, 0), _limbs(n, na, 9900, 1)
    C = oracle.intmatmul_pyint(A, B)
    g = np.random.default_rng(5)
    for _ in range(3):
        q = int(g.integers(2 ** 60, 2 ** 61)) | 1
        am = np.array([[oracle.limbs32_mod(A[i, l], q) for l in range(n)] for i in range(n)], dtype=object)
        bm = np.array([[oracle.limbs32_mod(B[i, l], q) for l in range(n)] for i in range(n)], dtype=object)
        want = am.dot(bm) % q
        got = np.array([[oracle.limbs32_mod(C[i, j], q) for j in range(n)] for i in range(n)], dtype=object)
        assert (got == want).all()


def test_integer_matrix_product_closed_forms():
    # all limbs 2^32 - 1: every entry is n (2^(32 na) - 1)^2 = n (2^(64 na) - 2^(32 na + 1) + 1)
    n, na = 4, 5
    full = np.full((n, n, na), 0xFFFFFFFF, dtype=np.uint32)
    C = oracle.intmatmul_pyint(full, full)
    want = n * (2 ** (64 * na) - 2 ** (32 * na + 1) + 1)
    for i in range(n):
        for j in range(n):
            assert int.from_bytes(C[i, j].astype("<u4").tobytes(), "little") == want
    # 1 x 1 reduces to the integer product; the identity matrix to a copy
    A, B = _limbs(1, 7, 9901, 0), _limbs(1, 7, 9901, 1)
    a16 = A[0, 0].astype("<u4").view("<u2")
    b16 = B[0, 0].astype("<u4").view("<u2")
    np.testing.assert_array_equal(oracle.intmatmul_pyint(A, B)[0, 0][:14], oracle.intmul_pyint(a16, b16))
    eye = np.zeros((3, 3, 2), dtype=np.uint32)
    for i in range(3):
        eye[i, i, 0] = 1
    M = _limbs(3, 2, 9902, 0)
    np.testing.assert_array_equal(oracle.intmatmul_pyint(M, eye)[:, :, :2], M)
