"""CPU-only checks of the C ABI library: it loads, exports every declared symbol,
and its host-side logic (number theory, argument checking, workspace sizes) agrees
with the oracle.  No call here reaches the GPU."""
import ctypes
import os
import re

import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import ntt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntt_mi355x.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ntt.LIB_PATH):
        pytest.fail("libntt_mi355x.so not built")
    return ntt.load()


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(ntt.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(ntt.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(raw, name), name


def test_strerror(lib):
    for code in range(-7, 1):
        assert lib.ntt_strerror(code)
    assert lib.ntt_strerror(0) == b"success"


def test_host_primality_matches_oracle(lib):
    import random
    r = random.Random(5)
    vals = list(range(0, 3000)) + [r.getrandbits(62) | 1 for _ in range(500)]
    vals += [998244353, 2013265921, 469762049, 167772161, 3215031751, 3825123056546413051]
    for n in vals:
        assert ntt.is_prime(n) == nt.is_prime(n), n


@pytest.mark.parametrize("p", [998244353, 2013265921, 469762049, 167772161, 97, 65537, 7340033])
def test_host_generator_matches_oracle(lib, p):
    assert ntt.smallest_generator(p) == nt.smallest_generator(p)


def test_host_generator_of_62bit_prime(lib):
    p = nt.largest_prime_below(62, 32)
    assert ntt.find_prime(62, 32) == p
    assert ntt.smallest_generator(p) == nt.smallest_generator(p)
    assert ntt.find_prime(31, 27) == 2013265921
    assert ntt.find_prime(30, 23) == 998244353


def _plan_rc(lib, p, g, log2n, flags=0):
    h = ctypes.c_void_p()
    return lib.ntt_plan_create(ctypes.byref(h), p, g, log2n, flags, None)


def test_plan_argument_errors(lib):
    assert _plan_rc(lib, 998244351, 0, 4) == ntt.NTT_ENOTPRIME
    assert _plan_rc(lib, 2, 0, 1) == ntt.NTT_EUNSUPPORTED
    assert _plan_rc(lib, 1 << 62, 0, 4) == ntt.NTT_EUNSUPPORTED
    assert _plan_rc(lib, 998244353, 0, 24) == ntt.NTT_ENOROOT      # 2-adic order 23
    assert lib.ntt_last_error() == b"2^24 does not divide p - 1 (2-adic order 23)"
    assert _plan_rc(lib, 998244353, 0, 27) == ntt.NTT_EUNSUPPORTED  # beyond 26
    assert _plan_rc(lib, 998244353, 2, 4) == ntt.NTT_ENOROOT       # 2 is not a generator
    assert _plan_rc(lib, 998244353, 0, 4, 0x80) == ntt.NTT_EINVAL
    assert lib.ntt_plan_create(None, 998244353, 0, 4, 0, None) == ntt.NTT_EINVAL
    assert lib.ntt_last_error() != b""


def test_polymul_argument_errors(lib):
    vp = ctypes.c_void_p
    one = vp(16)
    assert lib.polymul_modp(998244353, None, 0, None, 0, None, None, 0, None) == ntt.NTT_OK  # empty
    assert lib.polymul_modp(998244351, one, 4, one, 4, one, None, 0, None) == ntt.NTT_ENOTPRIME
    assert lib.polymul_modp(998244353, None, 4, one, 4, one, None, 0, None) == ntt.NTT_EINVAL
    # 2^23 + 1 coefficients need 2^24 | p - 1
    assert lib.polymul_modp(998244353, one, 1 << 22, one, (1 << 22) + 2, one, None, 0, None) == ntt.NTT_ENOROOT
    assert lib.polymul_modp(998244353, vp(2), 4, one, 4, one, None, 0, None) == ntt.NTT_EINVAL  # misaligned
    # multi-pass product without workspace
    assert lib.polymul_modp(998244353, one, 1 << 17, one, 1 << 17, one, None, 0, None) == ntt.NTT_ENOMEM


def test_polymul_noalloc_argument_errors(lib):
    one = ctypes.c_void_p(16)
    assert lib.polymul_modp_noalloc(998244353, None, 0, None, 0, None, None) == ntt.NTT_OK  # empty
    assert lib.polymul_modp_noalloc(998244351, one, 4, one, 4, one, None) == ntt.NTT_ENOTPRIME
    assert lib.polymul_modp_noalloc(998244353, one, 1 << 22, one, (1 << 22) + 2, one, None) == ntt.NTT_ENOROOT
    # two-pass scratch 2 N words: 2^23 32-bit words (N = 2^22) fit the fixed array, N = 2^23 does not
    assert lib.polymul_modp_noalloc(998244353, one, 1 << 22, one, (1 << 22) + 1, one, None) == ntt.NTT_ENOMEM
    assert b"more than the 33554432" in lib.ntt_last_error()
    p62 = nt.largest_prime_below(62, 32)
    assert lib.polymul_modp_noalloc(p62, one, 1 << 21, one, 2, one, None) == ntt.NTT_ENOMEM


def test_tft_argument_errors(lib):
    one = ctypes.c_void_p(16)
    assert lib.ntt_tft_workspace_bytes(None, 4) == 0
    assert lib.ntt_tft_forward(None, one, 4, one, 4, 1, 4, 4, None, 0, None) == ntt.NTT_EINVAL
    assert lib.ntt_tft_inverse(None, one, one, 4, 1, 4, 4, None, 0, None) == ntt.NTT_EINVAL
    assert b"plan is NULL" in lib.ntt_last_error()


def test_intmul_argument_errors(lib):
    vp = ctypes.c_void_p
    one = vp(16)
    assert lib.intmul_crt(one, 1 << 22, one, (1 << 22) + 2, one, None, 0, None) == ntt.NTT_EINVAL
    assert lib.intmul_crt(one, 10, one, 10, one, None, 0, None) == ntt.NTT_ENOMEM


def test_workspace_sizes(lib):
    ntt.tune_clear()  # built-in defaults: the 8192-point product is fused in one workgroup
    try:
        assert lib.polymul_workspace_bytes(998244353, 4096, 4096) == 0      # fused, no scratch
        ntt.tune_set("single.split.w32.L13", 1)                              # split: the 2 partials
        assert lib.polymul_workspace_bytes(998244353, 4096, 4096) == 4 * 8192
    finally:
        ntt.tune_clear()
        if os.path.exists(ntt.TUNE_FILE):
            ntt.tune_load(ntt.TUNE_FILE)
    assert lib.polymul_workspace_bytes(998244353, 1 << 20, 1 << 20) >= 2 * 4 * (1 << 21)
    assert lib.polymul_workspace_bytes(998244353, 0, 5) == 0
    assert lib.intmul_workspace_bytes(1 << 21, 1 << 21) >= 3 * 4 * ((1 << 22) - 1)
    assert lib.intmul_workspace_bytes(0, 5) == 0
    descs = (ntt.PolymulDesc * 2)()
    descs[0] = ntt.PolymulDesc(998244353, 16, 100, 16, 100, 16)
    descs[1] = ntt.PolymulDesc(2013265921, 16, 1 << 17, 16, 1 << 17, 16)
    ws = lib.polymul_batch_workspace_bytes(descs, 2)
    assert ws >= 2 * 4 * (1 << 18)


def test_intmul_chunk_bits_rule(lib):
    # section 5.3's rule with p1 p2 p3 ~ 2^86.02: h = 32 while 64 + ceil(log2(d + 1)) <= 86
    assert ntt.intmul_chunk_bits(1 << 21, 1 << 21) == 32        # d = 2^20 chunks of 32 bits: H = 85
    assert ntt.intmul_chunk_bits(2, 1) == 32
    big = (1 << 23) - 2                                          # d = 2^22 - 1 chunks: H = 64 + 22 = 86 < 86.02
    assert ntt.intmul_chunk_bits(big, big) == 32
    # d = 2^22 chunks: H = 64 + 23 = 87 is too many bits; 16-bit chunks: H = 32 + 23 fits
    assert ntt.intmul_chunk_bits((1 << 23) - 1, 1) == 16
    assert ntt.intmul_chunk_bits(1 << 24, 1 << 24) == 0          # no chunk size fits the transform lengths


def test_intmul32_argument_errors_and_sizes(lib):
    vp = ctypes.c_void_p
    one = vp(16)
    # coefficients could reach p1 p2 p3: min(na, nb) too large
    assert lib.intmul_crt32(one, 4300000, one, 4300000, one, None, 0, None) == ntt.NTT_EINVAL
    assert lib.intmul32_workspace_bytes(4300000, 4300000) == 0
    assert lib.intmul_crt32(one, 1 << 22, one, (1 << 22) + 2, one, None, 0, None) == ntt.NTT_EINVAL
    assert lib.intmul_crt32(one, 10, one, 10, one, None, 0, None) == ntt.NTT_ENOMEM
    assert lib.intmul_crt32(vp(2), 10, one, 10, one, None, 0, None) == ntt.NTT_EINVAL   # misaligned
    assert lib.intmul32_workspace_bytes(1 << 20, 1 << 20) >= 3 * 4 * ((1 << 21) - 1)


def test_polymatmul_argument_errors_and_sizes(lib):
    vp = ctypes.c_void_p
    one = vp(16)
    p = 469762049
    # Table 15's shape: 32 x 32 matrices, degrees < 2^15, transforms of 2^16 words
    assert lib.polymatmul_workspace_bytes(p, 32, 1 << 15) == 2 * 32 * 32 * (1 << 16) * 4
    assert lib.polymatmul_workspace_bytes(p, 0, 10) == 0
    assert lib.polymatmul_modp(p, 0, one, one, 10, one, None, 0, None) == ntt.NTT_OK
    assert lib.polymatmul_modp(p, 3, one, one, 0, one, None, 0, None) == ntt.NTT_OK
    assert lib.polymatmul_modp(p, 3, None, one, 10, one, None, 0, None) == ntt.NTT_EINVAL
    assert lib.polymatmul_modp(p, 3, vp(18), one, 10, one, None, 0, None) == ntt.NTT_EINVAL
    assert lib.polymatmul_modp(1000000000, 3, one, one, 10, one, None, 0, None) == ntt.NTT_ENOTPRIME
    assert lib.polymatmul_modp(4611685941117976577, 3, one, one, 10, one, None, 0, None) == ntt.NTT_EUNSUPPORTED
    assert lib.polymatmul_modp(p, 65, one, one, 10, one, None, 0, None) == ntt.NTT_EUNSUPPORTED
    # 7 * 2^20 + 1: degrees < 2^19 + 1 need transforms of 2^21 words
    assert lib.polymatmul_modp(7340033, 2, one, one, (1 << 19) + 1, one, None, 0, None) == ntt.NTT_ENOROOT
    assert lib.polymatmul_workspace_bytes(7340033, 2, (1 << 19) + 1) == 0
    assert lib.polymatmul_modp(p, 3, one, one, 10, one, None, 0, None) == ntt.NTT_ENOMEM


def test_f64_batch_argument_errors(lib):
    one = 16
    descs = (ntt.PolymulDesc * 1)()
    descs[0] = ntt.PolymulDesc(ntt.find_prime(50, 20), one, 8, one, 8, one)  # 2^49 < p < 2^50
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM
    p49 = ntt.find_prime(49, 20)
    p49b = ntt.find_prime(49, 25)
    descs[0] = ntt.PolymulDesc(p49b, one, 1 << 23, one, 1 << 23, one)        # transform 2^24
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EUNSUPPORTED
    assert lib.polymul_f64_batch_workspace_bytes(descs, 1) == 0
    descs[0] = ntt.PolymulDesc(p49, one, 1 << 15, one, 1 << 15, one)         # transform 2^16: two-pass
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM
    assert lib.polymul_f64_batch_workspace_bytes(descs, 1) >= (2 * 8) << 16
    descs[0] = ntt.PolymulDesc(1 << 50, one, 8, one, 8, one)                 # p >= 2^50
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EUNSUPPORTED
    descs[0] = ntt.PolymulDesc(p49, one, 8, one, 8, one)
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM
    assert lib.polymul_f64_batch_workspace_bytes(descs, 1) >= 64
    descs[0] = ntt.PolymulDesc(p49, one + 4, 8, one, 8, one)
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EINVAL
    descs[0] = ntt.PolymulDesc(p49 + 2, one, 8, one, 8, one)
    assert lib.polymul_f64_batch(descs, 1, None, 0, None) in (ntt.NTT_ENOTPRIME, ntt.NTT_ENOROOT)


def test_intmatmul_argument_errors_and_sizes(lib):
    one = ctypes.c_void_p(16)
    assert lib.intmatmul_crt32(0, one, one, 5, one, None, 0, None) == ntt.NTT_OK
    assert lib.intmatmul_crt32(65, one, one, 1, one, None, 0, None) == ntt.NTT_EUNSUPPORTED
    assert lib.intmatmul_crt32(64, one, one, 1 << 17, one, None, 0, None) == ntt.NTT_EINVAL   # n na > 2^22
    assert lib.intmatmul_crt32(2, one, one, 2, one, None, 0, None) == ntt.NTT_ENOMEM
    assert lib.intmatmul_crt32(2, ctypes.c_void_p(18), one, 2, one, None, 0, None) == ntt.NTT_EINVAL
    # the section's table: 32 x 32 entries of 2^15 chunks fit (32 2^15 (2^32 - 1)^2 < p1 p2 p3)
    assert lib.intmatmul32_workspace_bytes(32, 1 << 15) > 3 * 32 * 32 * ((1 << 16) - 1) * 4
    assert lib.intmatmul32_workspace_bytes(64, 1 << 17) == 0


def test_arith_apply_argument_errors(lib):
    one = ctypes.c_void_p(16)
    assert lib.ntt_arith_apply(9, 32, 998244353, one, one, one, 0, 0, one, 8, None) == ntt.NTT_EINVAL
    assert lib.ntt_arith_apply(0, 16, 998244353, one, one, one, 0, 0, one, 8, None) == ntt.NTT_EINVAL
    assert lib.ntt_arith_apply(0, 32, 998244352, one, one, one, 0, 0, one, 8, None) == ntt.NTT_EINVAL
    assert lib.ntt_arith_apply(0, 32, 2 ** 31 + 11, one, one, one, 0, 0, one, 8, None) == ntt.NTT_EUNSUPPORTED
    assert lib.ntt_arith_apply(0, 0, 2 ** 50 + 1, one, one, one, 0, 0, one, 8, None) == ntt.NTT_EUNSUPPORTED
    assert lib.ntt_arith_apply(0, 32, 998244353, one, one, None, 0, 0, one, 8, None) == ntt.NTT_EINVAL
    assert lib.ntt_arith_apply(2, 64, 998244353, ctypes.c_void_p(20), None, None, 0, 0, one, 8, None) == ntt.NTT_EINVAL
    assert lib.ntt_arith_apply(2, 64, 998244353, one, None, None, 0, 0, one, 0, None) == ntt.NTT_OK
