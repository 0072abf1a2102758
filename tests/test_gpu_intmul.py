"""GPU parity of the three-prime integer product (section 5.3), bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu


def _gpu_intmul(a, b):
    torch_cuda()
    return ntt.to_numpy(ntt.intmul(ntt.to_device(a), ntt.to_device(b)))


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 2), (2, 2), (3, 7), (64, 64), (1000, 999), (4096, 4096),
                                   (20000, 3), ((1 << 15), (1 << 15)), (70000, 65000), (70001, 65003)])
def test_intmul_against_python_int(na, nb):
    # (70000, 65000) and (70001, 65003): two-pass transforms whose column pass reads whole
    # runs of 4 limbs, or ends inside one (the per-run path of the column kernel)
    a = inputs.limbs16(na, inputs.CFG_TEST, na, 0)
    b = inputs.limbs16(nb, inputs.CFG_TEST, nb, 1)
    say("intmul na=%d nb=%d" % (na, nb))
    assert_equal_u(_gpu_intmul(a, b), oracle.intmul_pyint(a, b), "intmul")


def test_intmul_all_ones_closed_form():
    n = 50000
    ff = np.full(n, 0xFFFF, dtype=np.uint16)
    c = _gpu_intmul(ff, ff)
    v = int.from_bytes(c.astype("<u4").tobytes(), "little")
    assert v == (1 << (32 * n)) - (1 << (16 * n + 1)) + 1


def test_intmul_zero_length():
    torch_cuda()
    a = np.zeros(0, dtype=np.uint16)
    b = inputs.limbs16(5, inputs.CFG_TEST, 3)
    c = _gpu_intmul(a, b)
    assert c.size == 3 and np.all(c == 0)


def test_intmul_full_size_modular_checks():
    a, b = inputs.intmul_inputs()
    say("intmul full size 2^21 x 2^21 limbs")
    c = _gpu_intmul(a, b)
    assert c.size == 1 << 21
    rng = np.random.default_rng(9)
    for _ in range(6):
        q = int(rng.integers(1 << 60, 1 << 61)) | 1
        assert oracle.limbs32_mod(c, q) == oracle.limbs16_mod(a, q) * oracle.limbs16_mod(b, q) % q
    # low and high limbs against the exact product
    ref = oracle.intmul_pyint(a, b)
    assert_equal_u(c, ref, "intmul full size")


# ---------------------------------------------------------------- 32-bit chunks (section 5.3's h)

def _gpu_intmul32(a16, b16):
    torch_cuda()
    a32 = np.ascontiguousarray(a16).view("<u4")
    b32 = np.ascontiguousarray(b16).view("<u4")
    return ntt.to_numpy(ntt.intmul32(ntt.to_device(a32.astype(np.uint32)), ntt.to_device(b32.astype(np.uint32))))


@pytest.mark.parametrize("na,nb", [(2, 2), (2, 4), (6, 14), (128, 128), (2000, 1998), (8192, 8192),
                                   (40000, 6), ((1 << 15), (1 << 15)), (70000, 65000), (70002, 65006),
                                   (1 << 17, 1 << 16)])
def test_intmul32_against_python_int(na, nb):
    # na, nb 16-bit limbs (even): the same integers read as 32-bit chunks
    a = inputs.limbs16(na, inputs.CFG_TEST, 3000 + na, 0)
    b = inputs.limbs16(nb, inputs.CFG_TEST, 3000 + nb, 1)
    say("intmul32 na16=%d nb16=%d" % (na, nb))
    got = _gpu_intmul32(a, b)
    assert got.size == (na + nb) // 2
    assert_equal_u(got, oracle.intmul_pyint(a, b), "intmul32")


def test_intmul32_all_ones_closed_form():
    n = 30000  # 32-bit chunks of all ones
    torch_cuda()
    ff = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    c = ntt.to_numpy(ntt.intmul32(ntt.to_device(ff), ntt.to_device(ff)))
    v = int.from_bytes(c.astype("<u4").tobytes(), "little")
    assert v == (1 << (64 * n)) - (1 << (32 * n + 1)) + 1


def test_intmul32_equals_16_bit_path_full_size():
    # the integer product configuration (2^21 16-bit limbs each) through both chunk sizes
    a, b = inputs.intmul_inputs()
    say("intmul32 full size")
    c32 = _gpu_intmul32(a, b)
    assert_equal_u(c32, oracle.intmul_pyint(a, b), "32-bit chunks, full size, vs Python int")
    assert_equal_u(c32, _gpu_intmul(a, b), "32-bit chunks vs 16-bit limbs")
