"""polymul_modp_noalloc (the product without allocation: scratch in the library's
fixed device array) against polymul_modp (caller workspace) and the oracle, through
the C ABI.  Each case runs two no-allocation calls in a row on one stream, the second
on a smaller input, so the second call finds the first one's data in the shared
array: the fused kernel's park slice, the split path's partials, the two transformed
operands of the two-pass path (section 5.2's product in every case)."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)

# (p, (la, lb) of the first call, (la, lb) of the second, smaller call)
CASES = [
    (2013265921, (1 << 15, 1 << 15), (3000, 2000)),              # fused 2^16 (park slice), then 2^13
    (998244353, (4096, 4096), (1500, 700)),                      # the single product of 8192 points
    (998244353, (1 << 17, 1 << 17), ((1 << 16) + 5, 1000)),     # two-pass 2^18, then two-pass 2^17
    (P62, (1 << 19, 1 << 19), (5000, 4000)),                     # 64-bit words, two-pass 2^20 (16 MiB)
    (469762049, (1 << 21, 1 << 21), ((1 << 20) + 3, 12345)),     # two-pass 2^22: the whole 32 MiB array
]


def _operands(p, la, lb, seed):
    a = inputs.residues(p, la, inputs.CFG_TEST, seed, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, seed, 1)
    return a, b


@pytest.mark.parametrize("p,first,second", CASES)
def test_noalloc_matches_polymul_modp(p, first, second):
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    runs = []
    for k, (la, lb) in enumerate((first, second)):
        a, b = _operands(p, la, lb, 7700 + 10 * k + la % 7)
        da, db = ntt.to_device(a), ntt.to_device(b)
        say("noalloc: reference polymul_modp p=%d la=%d lb=%d" % (p, la, lb))
        ref = ntt.polymul(da, db, p, stream=stream)  # creates and caches the plan
        runs.append((a, b, da, db, ref))
    torch.cuda.synchronize()
    outs = []
    for a, b, da, db, ref in runs:
        out = torch.full_like(ref, -1)
        say("noalloc: polymul_modp_noalloc p=%d la=%d lb=%d" % (p, a.size, b.size))
        ntt.polymul_noalloc(da, db, p, out, stream=stream)
        outs.append(out)
    torch.cuda.synchronize()
    for (a, b, da, db, ref), out in zip(runs, outs):
        got = ntt.to_numpy(out)
        assert_equal_u(got, ntt.to_numpy(ref), "noalloc vs polymul_modp p=%d la=%d lb=%d" % (p, a.size, b.size))
        if a.size + b.size <= (1 << 19):
            assert_equal_u(got, oracle.polymul_ntt(a, b, p), "noalloc vs oracle p=%d la=%d lb=%d" % (p, a.size, b.size))


def test_noalloc_repeated_calls_keep_agreeing():
    """Several no-allocation calls of different paths in a row on one stream, each
    checked: every call rewrites what it reads of the array."""
    torch = torch_cuda()
    stream = torch.cuda.Stream()
    shapes = [(998244353, 1 << 17, 1 << 17), (2013265921, 1 << 15, 1 << 15), (998244353, 4096, 4096),
              (2013265921, 20000, 9000), (998244353, 100, 50)]
    refs = []
    for i, (p, la, lb) in enumerate(shapes):
        a, b = _operands(p, la, lb, 7900 + i)
        da, db = ntt.to_device(a), ntt.to_device(b)
        refs.append((p, da, db, ntt.polymul(da, db, p, stream=stream)))
    outs = []
    for p, da, db, ref in refs + refs[::-1]:
        out = torch.full_like(ref, -1)
        ntt.polymul_noalloc(da, db, p, out, stream=stream)
        outs.append((ref, out))
    torch.cuda.synchronize()
    for ref, out in outs:
        assert np.array_equal(ntt.to_numpy(out), ntt.to_numpy(ref))


def test_noalloc_refuses_missing_plan_and_large_products():
    torch = torch_cuda()
    q = 104857601  # 25 * 2^22 + 1: no product of this prime is made anywhere else in the tests
    a = ntt.to_device(inputs.residues(q, 3, inputs.CFG_TEST, 7990, 0))
    out = torch.empty(5, dtype=torch.int32, device="cuda")
    with pytest.raises(ntt.NTTError) as e:
        ntt.polymul_noalloc(a, a, q, out)
    assert e.value.code == ntt.NTT_EINVAL and "no cached plan" in str(e.value)
    big = torch.zeros(1 << 22, dtype=torch.int32, device="cuda")
    with pytest.raises(ntt.NTTError) as e:
        ntt.polymul_noalloc(big, big[:2], 998244353, big)
    assert e.value.code == ntt.NTT_ENOMEM
