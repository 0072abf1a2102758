"""Integer matrix product (section 5.3: Kronecker segmentation into 32-bit chunks,
polynomial matrix products modulo three primes, Garner and carries per entry) on the
GPU against Python's integers: every entry where that is quick, and for the
32 x 32 matrices of 2^20-bit integers (the section's table) sampled entries plus the
images of every entry modulo random 61-bit q."""
import numpy as np
import pytest

import oracle
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu


def _mats(n, na, item):
    A = inputs.limbs32(n * n * na, inputs.CFG_TEST, item, 0).reshape(n, n, na)
    B = inputs.limbs32(n * n * na, inputs.CFG_TEST, item, 1).reshape(n, n, na)
    return A, B


def _run(A, B):
    torch = torch_cuda()
    dA = ntt.to_device(A.reshape(-1)).reshape(A.shape)
    dB = ntt.to_device(B.reshape(-1)).reshape(B.shape)
    C = ntt.intmatmul32(dA, dB)
    torch.cuda.synchronize()
    return ntt.to_numpy(C.reshape(-1)).reshape(C.shape).astype(np.uint32)


@pytest.mark.parametrize("n,na", [(1, 1), (1, 7), (2, 3), (3, 100), (5, 1000), (2, 5000), (8, 300), (64, 2),
                                  (33, 17), (4, 4097)])
def test_intmatmul_equals_python_integers(n, na):
    say("intmatmul n=%d na=%d" % (n, na))
    A, B = _mats(n, na, 9300 + n * 11 + na)
    got = _run(A, B)
    assert_equal_u(got.reshape(-1), oracle.intmatmul_pyint(A, B).reshape(-1), "intmatmul n=%d na=%d" % (n, na))


def test_intmatmul_all_ones_closed_form():
    n, na = 6, 1000
    full = np.full((n, n, na), 0xFFFFFFFF, dtype=np.uint32)
    got = _run(full, full)
    want = n * (2 ** (64 * na) - 2 ** (32 * na + 1) + 1)
    wl = np.frombuffer(want.to_bytes(4 * (2 * na + 1), "little"), dtype="<u4")
    for i in range(n):
        for j in range(n):
            assert_equal_u(got[i, j], wl, "all ones (%d, %d)" % (i, j))


def test_intmatmul_table_configuration():
    """32 x 32 matrices of integers of 32 x 2^15 bits."""
    n, na = 32, 1 << 15
    say("intmatmul 32 x 32, 2^15 limbs")
    A, B = _mats(n, na, 9399)
    C = _run(A, B)
    for (i, j) in [(0, 0), (31, 31), (7, 19)]:
        v = oracle.intmatmul_entry_pyint(A, B, i, j)
        wl = np.frombuffer(v.to_bytes(4 * (2 * na + 1), "little"), dtype="<u4")
        assert_equal_u(C[i, j], wl, "entry (%d, %d)" % (i, j))
    g = np.random.default_rng(17)
    q = int(g.integers(2 ** 60, 2 ** 61)) | 1
    am = np.array([[oracle.limbs32_mod(A[i, l], q) for l in range(n)] for i in range(n)], dtype=object)
    bm = np.array([[oracle.limbs32_mod(B[i, l], q) for l in range(n)] for i in range(n)], dtype=object)
    want = am.dot(bm) % q
    got = np.array([[oracle.limbs32_mod(C[i, j], q) for j in range(n)] for i in range(n)], dtype=object)
    assert (got == want).all(), "images modulo q = %d" % q


def test_intmatmul_errors():
    torch = torch_cuda()
    L = ntt.load()
    x = torch.zeros(16, dtype=torch.int32, device="cuda")
    assert L.intmatmul_crt32(65, ntt._ptr(x), ntt._ptr(x), 1, ntt._ptr(x), None, 0, None) == ntt.NTT_EUNSUPPORTED
    assert L.intmatmul_crt32(64, ntt._ptr(x), ntt._ptr(x), 1 << 17, ntt._ptr(x), None, 0, None) == ntt.NTT_EINVAL
    assert L.intmatmul_crt32(2, ntt._ptr(x), ntt._ptr(x), 2, ntt._ptr(x), None, 0, None) == ntt.NTT_ENOMEM
    assert L.intmatmul32_workspace_bytes(64, 1 << 17) == 0
