"""Polynomial matrix product (section 5.2) on the GPU against the oracle: every
coefficient where the schoolbook oracle finishes in seconds, and at larger sizes --
up to the 32 x 32, degree < 2^15 configuration of the section's table -- sampled
coefficients plus the evaluation identity C(x) = A(x) B(x) over F_p at random points."""
import numpy as np
import pytest

import oracle
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu


def _mats(p, n, d, item):
    A = inputs.residues(p, n * n * d, inputs.CFG_TEST, item, 0).reshape(n, n, d)
    B = inputs.residues(p, n * n * d, inputs.CFG_TEST, item, 1).reshape(n, n, d)
    return A, B


def _run(A, B, p):
    torch = torch_cuda()
    dA = ntt.to_device(A.reshape(-1)).reshape(A.shape)
    dB = ntt.to_device(B.reshape(-1)).reshape(B.shape)
    C = ntt.polymatmul(dA, dB, p)
    torch.cuda.synchronize()
    return ntt.to_numpy(C.reshape(-1)).reshape(C.shape)


def _check_sampled(A, B, C, p, samples, seed):
    n, d = A.shape[0], A.shape[2]
    g = np.random.default_rng(seed)
    picks = [(0, 0, 0), (n - 1, n - 1, 2 * d - 2), (n - 1, 0, d - 1), (0, n - 1, d)]
    picks += [(int(g.integers(n)), int(g.integers(n)), int(g.integers(2 * d - 1))) for _ in range(samples)]
    for (i, j, k) in picks:
        if k >= 2 * d - 1:
            continue
        want = oracle.polymatmul_coeff(A, B, p, i, j, k)
        assert int(C[i, j, k]) == want, ("coefficient", i, j, k, int(C[i, j, k]), want)
    # C(x) = A(x) B(x) over F_p at random points (Schwartz-Zippel: false accept <= 2d / p)
    for _ in range(2):
        x = np.array([int(g.integers(1, p))], dtype=np.uint64)
        ea = np.array([[int(oracle.horner_many(A[i, l], p, x)[0]) for l in range(n)] for i in range(n)], dtype=object)
        eb = np.array([[int(oracle.horner_many(B[l, j], p, x)[0]) for j in range(n)] for l in range(n)], dtype=object)
        want = ea.dot(eb) % p
        got = np.array([[int(oracle.horner_many(C[i, j], p, x)[0]) for j in range(n)] for i in range(n)], dtype=object)
        assert (got == want).all(), "evaluation identity at x = %d" % int(x[0])


EXACT = [
    (469762049, 1, 1), (469762049, 2, 2), (469762049, 1, 4096), (469762049, 3, 100), (998244353, 4, 257),
    (2013265921, 5, 300), (7340033, 8, 64), (469762049, 13, 40), (469762049, 64, 8), (469762049, 33, 30),
    (469762049, 9, 700), (2013265921, 2, 4097), (998244353, 2, 5000), (469762049, 17, 3),
    # n = 32: the section's largest matrices, exact at small degrees (31-bit and small primes)
    (469762049, 32, 40), (2013265921, 32, 9), (7340033, 32, 3), (998244353, 32, 2), (469762049, 32, 1),
]


@pytest.mark.parametrize("p,n,d", EXACT)
def test_polymatmul_equals_oracle(p, n, d):
    say("polymatmul p=%d n=%d d=%d" % (p, n, d))
    A, B = _mats(p, n, d, 9000 + n * 7 + d)
    got = _run(A, B, p)
    want = oracle.polymatmul(A, B, p)
    assert_equal_u(got.reshape(-1), want.reshape(-1), "polymatmul p=%d n=%d d=%d" % (p, n, d))


@pytest.mark.parametrize("p,n,d", [(469762049, 4, 20000), (998244353, 6, 9000), (2013265921, 3, 40000)])
def test_polymatmul_two_pass_sampled(p, n, d):
    say("polymatmul two-pass p=%d n=%d d=%d" % (p, n, d))
    A, B = _mats(p, n, d, 9050 + n)
    C = _run(A, B, p)
    _check_sampled(A, B, C, p, 48, n * d)


def test_polymatmul_table_configuration():
    """32 x 32 matrices, degrees < 2^15, p = 469762049 (the section's table, largest n)."""
    p, n, d = 469762049, 32, 1 << 15
    say("polymatmul 32 x 32, d = 2^15")
    A, B = _mats(p, n, d, 9099)
    C = _run(A, B, p)
    assert C.shape == (n, n, 2 * d - 1)
    _check_sampled(A, B, C, p, 96, 32768)


def test_polymatmul_edge_values_and_identity():
    torch = torch_cuda()
    p, n, d = 469762049, 6, 1000
    full = np.full((n, n, d), p - 1, dtype=np.uint32)
    got = _run(full, full, p)
    k = np.arange(2 * d - 1)
    terms = np.minimum(k, 2 * d - 2 - k) + 1
    want = np.array([n * int(t) * (p - 1) ** 2 % p for t in terms], dtype=np.uint64)
    for i in range(n):
        for j in range(n):
            assert_equal_u(got[i, j], want, "all p-1 entry (%d, %d)" % (i, j))
    A, _ = _mats(p, n, d, 9111)
    eye = np.zeros((n, n, d), dtype=np.uint32)
    for i in range(n):
        eye[i, i, 0] = 1
    got = _run(A, eye, p)
    assert_equal_u(got[:, :, :d].reshape(-1), A.reshape(-1), "A times identity")
    assert not got[:, :, d:].any()
    torch.cuda.synchronize()


def test_polymatmul_workspace_reuse_and_stream():
    """Two products in a row through one caller-owned workspace on a side stream."""
    torch = torch_cuda()
    s = torch.cuda.Stream()
    p = 998244353
    L = ntt.load()
    ws = torch.empty(L.polymatmul_workspace_bytes(p, 5, 3000), dtype=torch.uint8, device="cuda")
    for (n, d, item) in [(5, 3000, 9120), (3, 700, 9121)]:
        A, B = _mats(p, n, d, item)
        dA = ntt.to_device(A.reshape(-1)).reshape(A.shape)
        dB = ntt.to_device(B.reshape(-1)).reshape(B.shape)
        torch.cuda.synchronize()
        C = torch.empty((n, n, 2 * d - 1), dtype=torch.int32, device="cuda")
        ntt.polymatmul(dA, dB, p, out=C, stream=s, workspace=ws)
        s.synchronize()
        assert_equal_u(ntt.to_numpy(C.reshape(-1)), oracle.polymatmul(A, B, p).reshape(-1), "n=%d d=%d" % (n, d))
