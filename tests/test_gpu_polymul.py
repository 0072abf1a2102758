"""GPU parity of the polynomial product (section 5.2) against the CPU oracle,
bit-exact, through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)
PRIMES = [998244353, 2013265921, 469762049, 167772161, P62]


def _gpu_polymul(a, b, p):
    torch_cuda()
    c = ntt.polymul(ntt.to_device(a), ntt.to_device(b), p)
    return ntt.to_numpy(c)


def test_polymul_8k_config_exact():
    p, a, b = inputs.polymul_8k_inputs()
    say("polymul 8k p=%d" % p)
    c = _gpu_polymul(a, b, p)
    assert c.size == 8191
    assert_equal_u(c, oracle.polymul_schoolbook(a, b, p), "polymul 8k")


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("la,lb", [(1, 1), (1, 2), (2, 2), (3, 5), (16, 17), (100, 29), (512, 513), (1000, 1000),
                                   (2048, 2049), (4096, 4096), (4097, 4096)])
def test_polymul_small_sizes(p, la, lb):
    a = inputs.residues(p, la, inputs.CFG_TEST, la, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, lb, 1)
    say("polymul p=%d la=%d lb=%d" % (p, la, lb))
    assert_equal_u(_gpu_polymul(a, b, p), oracle.polymul_ntt(a, b, p), "polymul")


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("la,lb", [(8192, 8192), (8193, 8192), (1 << 14, 3), (16384, 16385), (1 << 15, 1 << 15),
                                   ((1 << 15) + 1, 1 << 15), (1 << 16, 1 << 16), (100000, 31073)])
def test_polymul_medium_and_multipass(p, la, lb):
    lc = la + lb - 1
    if lc > (1 << nt.two_adic(p)[1]):
        pytest.skip("length beyond the prime's 2-adic order")
    a = inputs.residues(p, la, inputs.CFG_TEST, la, 2)
    b = inputs.residues(p, lb, inputs.CFG_TEST, lb, 3)
    say("polymul p=%d la=%d lb=%d" % (p, la, lb))
    assert_equal_u(_gpu_polymul(a, b, p), oracle.polymul_ntt(a, b, p), "polymul")


@pytest.mark.parametrize("p", [998244353, 2013265921, P62])
@pytest.mark.parametrize("kind", ["zeros", "pm1", "alternating", "ones"])
def test_polymul_structured(p, kind):
    for n in (7, 4096, 20000):
        a = inputs.structured(kind, p, n)
        b = inputs.structured("pm1" if kind != "zeros" else "ones", p, n + 3)
        say("polymul structured %s p=%d n=%d" % (kind, p, n))
        assert_equal_u(_gpu_polymul(a, b, p), oracle.polymul_ntt(a, b, p), "polymul structured")


def test_polymul_empty():
    torch = torch_cuda()
    a = ntt.to_device(np.zeros(0, dtype=np.uint32))
    b = ntt.to_device(np.arange(5, dtype=np.uint32))
    c = ntt.polymul(a, b, 998244353)
    assert c.numel() == 0


def test_polymul_errors_on_device():
    torch_cuda()
    a = ntt.to_device(np.ones((1 << 22) + 1, dtype=np.uint32))
    with pytest.raises(ntt.NTTError) as e:
        ntt.polymul(a, a, 998244353)  # 2^23 + 1 coefficients exceed the 2-adic order 23
    assert e.value.code == ntt.NTT_ENOROOT


@pytest.mark.parametrize("items,p", [(8, 2013265921), (3, 998244353), (5, P62)])
def test_polymul_batch_rows(items, p):
    torch = torch_cuda()
    length = 1 << 15 if p < (1 << 62) and p != P62 else 1 << 14
    _, A, B = inputs.polymul_batch_inputs(items, length, p)
    say("polymul rows items=%d L=%d p=%d" % (items, length, p))
    C = ntt.to_numpy(ntt.polymul_rows(ntt.to_device(A), ntt.to_device(B), p))
    for i in range(items):
        assert_equal_u(C[i], oracle.polymul_ntt(A[i], B[i], p), "batch item %d" % i)


def test_polymul_batch_mixed_primes_and_sizes():
    torch = torch_cuda()
    specs = [(998244353, 5, 9), (2013265921, 4096, 4096), (P62, 1000, 300), (469762049, 1 << 15, 1 << 15),
             (167772161, 1, 1), (2013265921, 70000, 70000), (P62, 1 << 14, (1 << 14) + 1), (998244353, 0, 7)]
    pairs, ref = [], []
    for i, (p, la, lb) in enumerate(specs):
        a = inputs.residues(p, la, inputs.CFG_TEST, 1000 + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 1000 + i, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        ref.append(oracle.polymul_ntt(a, b, p) if la and lb else np.zeros(0, dtype=np.uint64))
    say("polymul batch mixed")
    outs = ntt.polymul_batch(pairs, [s[0] for s in specs])
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert_equal_u(ntt.to_numpy(o), r, "mixed item %d" % i)


# TFT truncation in the fused batch kernel: 2^16-point products with lc <= 3 * 2^14
# compute 3 of their 4 sub-problems and complete the fourth from the zero coefficients
@pytest.mark.parametrize("la,lb", [(16385, 16385), (20000, 18000), (24576, 24576), (24577, 24576), (24577, 24577),
                                   (40000, 2), (2, 49000)])
def test_fused_truncated_products(la, lb):
    torch_cuda()
    p = 2013265921
    pairs, outs, want = [], [], []
    for k in range(3):
        a = inputs.residues(p, la, inputs.CFG_TEST, 1700 + k, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 1700 + k, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        want.append(oracle.polymul_ntt(a, b, p, 31))
    say("fused batch truncated products la=%d lb=%d" % (la, lb))
    got = ntt.polymul_batch(pairs, [p] * 3)
    for k in range(3):
        assert_equal_u(ntt.to_numpy(got[k]), want[k], "fused truncated product %d" % k)


# The same truncation in the 64-bit-word fused kernel (2^15-point products, sub-problems
# of 2^13): lc <= 3 * 2^13 computes 3 of the 4 sub-problems
@pytest.mark.parametrize("la,lb", [(8193, 8193), (10000, 9000), (12288, 12288), (12289, 12288), (12289, 12289),
                                   (20000, 2), (2, 24000)])
def test_fused_truncated_products_64bit(la, lb):
    torch_cuda()
    p = P62
    pairs, want = [], []
    for k in range(2):
        a = inputs.residues(p, la, inputs.CFG_TEST, 1750 + k, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 1750 + k, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        want.append(oracle.polymul_ntt(a, b, p))
    say("64-bit fused batch truncated products la=%d lb=%d" % (la, lb))
    got = ntt.polymul_batch(pairs, [p] * 2)
    for k in range(2):
        assert_equal_u(ntt.to_numpy(got[k]), want[k], "64-bit fused truncated product %d" % k)
