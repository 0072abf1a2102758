"""Products mod p computed with residues held in doubles (section 3: Function 16 for
products, Function 17 for sums) against the oracle's integer schoolbook product, and
against the 64-bit integer path on the same inputs."""
import numpy as np
import pytest

import oracle
from oracle import numtheory
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P48 = numtheory.largest_prime_below(48, 20)   # lazy ranges (operands below 4p)
P49 = numtheory.largest_prime_below(49, 20)   # operands below 2p
SHAPES = [(1, 1), (2, 3), (100, 37), (1000, 1000), (4096, 4096), (5000, 11), (3000, 9000), (1 << 14, 1 << 14),
          (16383, 2),
          # 2^15-point products with lc <= 3 * 2^13: 3 of 4 sub-problems (TFT truncation)
          (8193, 8193), (12288, 12289), (20000, 2)]


def _f64(x, torch):
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("p", [998244353, P48, P49])
def test_f64_products_equal_oracle(p):
    torch = torch_cuda()
    pairs, outs, want = [], [], []
    for i, (la, lb) in enumerate(SHAPES):
        a = inputs.residues(p, la, inputs.CFG_TEST, 6100 + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 6100 + i, 1)
        pairs.append((_f64(a, torch), _f64(b, torch)))
        outs.append(torch.empty(la + lb - 1, dtype=torch.float64, device="cuda"))
        want.append(oracle.polymul_schoolbook(a, b, p))
    L = ntt.load()
    descs = (ntt.PolymulDesc * len(pairs))()
    for i, ((a, b), c) in enumerate(zip(pairs, outs)):
        descs[i] = ntt.PolymulDesc(p, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), c.data_ptr())
    ws = torch.empty(max(L.polymul_f64_batch_workspace_bytes(descs, len(pairs)), 1), dtype=torch.uint8, device="cuda")
    say("f64 batch p=%d" % p)
    ntt._check(L.polymul_f64_batch(descs, len(pairs), ntt._ptr(ws), ws.numel(), None), "polymul_f64_batch")
    torch.cuda.synchronize()
    for (la, lb), c, w in zip(SHAPES, outs, want):
        got = c.cpu().numpy()
        assert (got == np.floor(got)).all() and (got >= 0).all() and (got < p).all()
        assert_equal_u(got.astype(np.uint64), w, "f64 p=%d %dx%d" % (p, la, lb))


def test_f64_rows_match_integer_path():
    """A batch of 64 rows of length 2^14 mod a 49-bit prime: the FP64 and the 64-bit
    integer kernels give the same residues; two rows also against the oracle."""
    torch = torch_cuda()
    p, items, n = P49, 64, 1 << 14
    _, A, B = inputs.polymul_batch_inputs(items, n, p)
    dA64, dB64 = ntt.to_device(A), ntt.to_device(B)
    C64 = ntt.polymul_rows(dA64, dB64, p)
    Af, Bf = dA64.double(), dB64.double()  # exact: residues below 2^49
    Cf = ntt.polymul_f64_rows(Af, Bf, p)
    torch.cuda.synchronize()
    say("f64 rows vs integer rows")
    gi = ntt.to_numpy(C64.reshape(-1))
    gf = Cf.cpu().numpy().reshape(-1).astype(np.uint64)
    assert_equal_u(gf, gi, "f64 vs u64 rows")
    for r in (0, items - 1):
        assert_equal_u(Cf[r].cpu().numpy().astype(np.uint64), oracle.polymul_schoolbook(A[r], B[r], p), "row %d" % r)
    # the reusable handle gives the same, twice in a row
    Cb = torch.full_like(Cf, -1.0)
    bt = ntt.Batch.rows(Af, Bf, Cb, p, f64=True)
    for _ in range(2):
        Cb.fill_(-1.0)
        bt()
        torch.cuda.synchronize()
        assert torch.equal(Cb, Cf)
    bt.close()


def test_f64_errors():
    torch = torch_cuda()
    L = ntt.load()
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    c = torch.zeros(15, dtype=torch.float64, device="cuda")
    descs = (ntt.PolymulDesc * 1)()
    big = 63 * 2 ** 44 + 1  # prime just below 2^50: operands below 2p would exceed Function 16's bound
    descs[0] = ntt.PolymulDesc(big, a.data_ptr(), 8, a.data_ptr(), 8, c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EUNSUPPORTED
    long_a = torch.zeros(1 << 15, dtype=torch.float64, device="cuda")
    long_c = torch.zeros((1 << 16) - 1, dtype=torch.float64, device="cuda")
    descs[0] = ntt.PolymulDesc(P49, long_a.data_ptr(), 1 << 15, long_a.data_ptr(), 1 << 15, long_c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EUNSUPPORTED  # transform 2^16 > 2^15
    descs[0] = ntt.PolymulDesc(P49, a.data_ptr(), 8, a.data_ptr(), 8, c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM
    descs[0] = ntt.PolymulDesc(P49, a.data_ptr() + 4, 7, a.data_ptr(), 8, c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EINVAL
