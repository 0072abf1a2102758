"""Residues held in doubles (section 3: Function 16 for products, Function 17 for sums):
products against the oracle's integer schoolbook and transform products, and against the
64-bit integer path on the same inputs; transforms of NTT_FP64 plans against the
oracle's textbook transform.  Primes below 2^48 (lazy ranges), between 2^48 and 2^49, and
between 2^49 and 2^50 (multiplicands reduced before each product)."""
import numpy as np
import pytest

import oracle
from oracle import numtheory
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P48 = numtheory.largest_prime_below(48, 20)   # lazy ranges (operands below 4p)
P49 = numtheory.largest_prime_below(49, 20)   # operands below 2p
P50 = numtheory.largest_prime_below(50, 20)   # multiplicands reduced to [0, p) first
P50B = 63 * 2 ** 44 + 1                        # 2^49 < p < 2^50, roots of order up to 2^44
SHAPES = [(1, 1), (2, 3), (100, 37), (1000, 1000), (4096, 4096), (5000, 11), (3000, 9000), (1 << 14, 1 << 14),
          (16383, 2),
          # 2^15-point products with lc <= 3 * 2^13: 3 of 4 sub-problems (TFT truncation)
          (8193, 8193), (12288, 12289), (20000, 2)]


def _f64(x, torch):
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("p", [998244353, P48, P49, P50, P50B])
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
    descs[0] = ntt.PolymulDesc(2 ** 50 + 55, a.data_ptr(), 8, a.data_ptr(), 8, c.data_ptr())  # p >= 2^50
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EUNSUPPORTED
    long_a = torch.zeros(1 << 15, dtype=torch.float64, device="cuda")
    long_c = torch.zeros((1 << 16) - 1, dtype=torch.float64, device="cuda")
    descs[0] = ntt.PolymulDesc(P49, long_a.data_ptr(), 1 << 15, long_a.data_ptr(), 1 << 15, long_c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM  # two-pass 2^16: needs workspace
    descs[0] = ntt.PolymulDesc(P49, a.data_ptr(), 8, a.data_ptr(), 8, c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_ENOMEM
    descs[0] = ntt.PolymulDesc(P49, a.data_ptr() + 4, 7, a.data_ptr(), 8, c.data_ptr())
    assert L.polymul_f64_batch(descs, 1, None, 0, None) == ntt.NTT_EINVAL


# two-pass products (transforms above 2^15: columns, twiddles, rows, columns)
LONG_SHAPES = [(1 << 15, 1 << 15), (20000, 30001), (40000, 3), (1, 70000), ((1 << 16) + 3, 50000), (200001, 300000)]


@pytest.mark.parametrize("p", [P48, P49, P50])
def test_f64_two_pass_products_equal_oracle(p):
    torch = torch_cuda()
    L = ntt.load()
    pairs, outs, want = [], [], []
    for i, (la, lb) in enumerate(LONG_SHAPES):
        a = inputs.residues(p, la, inputs.CFG_TEST, 6300 + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 6300 + i, 1)
        pairs.append((_f64(a, torch), _f64(b, torch)))
        outs.append(torch.full((la + lb - 1,), -1.0, dtype=torch.float64, device="cuda"))
        want.append(oracle.polymul_ntt(a, b, p))
    descs = (ntt.PolymulDesc * len(pairs))()
    for i, ((a, b), c) in enumerate(zip(pairs, outs)):
        descs[i] = ntt.PolymulDesc(p, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), c.data_ptr())
    ws = torch.empty(max(L.polymul_f64_batch_workspace_bytes(descs, len(pairs)), 1), dtype=torch.uint8, device="cuda")
    say("f64 two-pass batch p=%d" % p)
    ntt._check(L.polymul_f64_batch(descs, len(pairs), ntt._ptr(ws), ws.numel(), None), "polymul_f64_batch")
    torch.cuda.synchronize()
    for (la, lb), c, w in zip(LONG_SHAPES, outs, want):
        got = c.cpu().numpy()
        assert (got == np.floor(got)).all() and (got >= 0).all() and (got < p).all()
        assert_equal_u(got.astype(np.uint64), w, "f64 two-pass p=%d %dx%d" % (p, la, lb))
    # the reusable handle (its two-pass items included) gives the same, twice in a row
    bt = ntt.Batch((descs, len(pairs)), f64=True)
    for _ in range(2):
        for c in outs:
            c.fill_(-1.0)
        bt()
        torch.cuda.synchronize()
        for (la, lb), c, w in zip(LONG_SHAPES, outs, want):
            assert_equal_u(c.cpu().numpy().astype(np.uint64), w, "f64 handle p=%d %dx%d" % (p, la, lb))
    bt.close()


def _f64_plan(p, log2n, flags):
    plan = ntt.Plan(p, log2n, 0, flags | ntt.NTT_FP64)
    return plan, numtheory.root_of_unity(p, 1 << log2n, plan.info.g)


@pytest.mark.parametrize("p", [998244353, P48, P49, P50B])
@pytest.mark.parametrize("log2n", [0, 1, 3, 5, 10, 12, 13, 14, 15, 16, 18])
@pytest.mark.parametrize("bitrev", [False, True])
def test_f64_transforms_exact(p, log2n, bitrev):
    torch = torch_cuda()
    n = 1 << log2n
    batch = 3 if log2n <= 14 else 1
    flags = (ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN) if bitrev else 0
    plan, w = _f64_plan(p, log2n, flags)
    x = np.stack([inputs.residues(p, n, inputs.CFG_TEST, 6400 + log2n, i) for i in range(batch)])
    say("f64 ntt p=%d log2n=%d bitrev=%s passes=%d" % (p, log2n, bitrev, plan.info.passes))
    X = plan.forward(_f64(x.reshape(-1), torch), batch=batch)
    got = X.cpu().numpy().reshape(batch, n)
    assert (got == np.floor(got)).all() and (got >= 0).all() and (got < p).all()
    for i in range(batch):
        ref = oracle.ntt(x[i], p, w)
        if bitrev:
            ref = oracle.tft_order(ref)
        assert_equal_u(got[i].astype(np.uint64), ref, "f64 forward vec %d" % i)
    back = plan.inverse(X, batch=batch).cpu().numpy()
    assert_equal_u(back.astype(np.uint64), x.reshape(-1), "f64 inverse(forward)")
    plan.close()


@pytest.mark.parametrize("p,log2n", [(P49, 20), (P50B, 23)])
def test_f64_large_transform_spot_checks_and_integer_path(p, log2n):
    """Long FP64 transforms: spot checks by evaluation, the round trip, and equality
    with the 64-bit integer plan of the same prime and generator."""
    torch = torch_cuda()
    n = 1 << log2n
    flags = ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN
    plan, w = _f64_plan(p, log2n, flags)
    iplan = ntt.Plan(p, log2n, plan.info.g, flags)
    x = inputs.residues(p, n, inputs.CFG_TEST, 6500 + log2n)
    say("f64 ntt large p=%d log2n=%d passes=%d" % (p, log2n, plan.info.passes))
    X = plan.forward(_f64(x, torch))
    Xh = X.cpu().numpy().astype(np.uint64)
    idx = np.random.default_rng(log2n).integers(0, n, size=48)
    pts = [pow(w, oracle.bitrev(int(i), log2n), p) for i in idx]
    assert_equal_u(Xh[idx], oracle.horner_many(x, p, pts), "f64 forward spot checks")
    assert_equal_u(Xh, ntt.to_numpy(iplan.forward(ntt.to_device(x))), "f64 vs 64-bit integer plan")
    assert_equal_u(plan.inverse(X).cpu().numpy().astype(np.uint64), x, "f64 roundtrip")
    torch.cuda.synchronize()
    plan.close()
    iplan.close()


def test_f64_plan_errors():
    torch_cuda()
    with pytest.raises(ntt.NTTError) as e:
        ntt.Plan(ntt.find_prime(51, 20), 10, 0, ntt.NTT_FP64)  # a prime above 2^50
    assert e.value.code == ntt.NTT_EUNSUPPORTED
    with pytest.raises(ntt.NTTError) as e:
        ntt.Plan(P49, 10, 0, ntt.NTT_FP64 | ntt.NTT_VALIDATE)
    assert e.value.code == ntt.NTT_EUNSUPPORTED
