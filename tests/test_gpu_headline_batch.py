"""The batched product at its full size, every item against the oracle (section 5.2's
polynomial product: two forward transforms, the entry-wise product, one inverse).

The 1024 products mod 2013265921 of length-2^15 operands run exactly as the benchmark
launches them (one reusable batch handle over row-major operand matrices), and every
product of the batch is compared bit-exactly with the oracle's transform product.  A
second batch holds more products than the chip has workgroups for that size class,
with shapes that differ from one product of a workgroup to its next (full-length,
truncated, 2^14- and 2^15-point products, products with one operand longer than
half the transform, three primes), so that the persistent item loop and the reuse of
each workgroup's park slice across items are checked too.  Both kernels of 2^16-point
products run every case: four sub-problems of 2^14 points, and two of 2^15."""
import numpy as np
import pytest

import oracle
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, oracle_many, say, torch_cuda

pytestmark = pytest.mark.gpu

P = inputs.P_2013


@pytest.fixture(params=[0, 1], ids=["subproblems_2^14", "subproblems_2^15"])
def m15(request):
    """The two kernels of 2^16-point products: four sub-problems of 2^14 points (class
    3), or two of 2^15 (class 4, tuning choice fused.m15.w32)."""
    ntt.tune_set("fused.m15.w32", request.param)
    yield request.param
    ntt.tune_set("fused.m15.w32", 0)


def test_headline_batch_every_item(m15):
    torch = torch_cuda()
    items, L = 1024, 1 << 15
    say("headline batch: %d products mod %d, operands of %d, fused.m15.w32=%d" % (items, P, L, m15))
    _, A, B = inputs.polymul_batch_inputs(items, L, P)
    dA, dB = ntt.to_device(A), ntt.to_device(B)
    dC = torch.full((items, 2 * L - 1), -1, dtype=torch.int32, device="cuda")
    batch = ntt.Batch.rows(dA, dB, dC, P)
    stream = torch.cuda.Stream()
    batch(stream)
    torch.cuda.synchronize()
    C = ntt.to_numpy(dC)
    say("headline batch: oracle on %d items" % items)
    want = oracle_many(oracle.polymul_ntt, [(A[i], B[i], P, 31) for i in range(items)])
    for i in range(items):
        assert_equal_u(C[i], want[i], "headline batch item %d" % i)
    # a second launch of the same handle (the park slices hold the first launch's data)
    dC.fill_(-1)
    batch(stream)
    torch.cuda.synchronize()
    C2 = ntt.to_numpy(dC)
    assert np.array_equal(C2, C), "second launch of the batch handle differs"
    batch.close()


def _long_short(g):
    la = int(g.integers(32769, 65536))
    lb = int(g.integers(1, 65538 - la))
    return (la, lb) if g.integers(0, 2) else (lb, la)


def _mixed_shapes(count: int, seed: int):
    """(p, la, lb) per item: class-3 products of 2^14, 2^15 and 2^16 points, full and
    truncated, under three primes, drawn so that consecutive items of one workgroup
    (items w, w + G, w + 2G, ...) take different shapes."""
    g = inputs.rng(inputs.CFG_TEST, seed)
    primes = [inputs.P_2013, inputs.P_998, inputs.P_469]
    kinds = [
        lambda: (1 << 15, 1 << 15),                              # 2^16 points, all 4 sub-problems
        lambda: (int(g.integers(20000, 24577)), int(g.integers(16385, 24577))),  # 2^16 points, lc <= 3 * 2^14
        lambda: (int(g.integers(24577, 32769)), int(g.integers(24577, 32769))),  # 2^16 points, lc > 3 * 2^14
        lambda: (int(g.integers(12289, 20000)), int(g.integers(4097, 8193))),    # 2^15 points
        lambda: (int(g.integers(4097, 8193)), int(g.integers(4097, 8193))),      # 2^14 points
        lambda: _long_short(g),                                  # 2^16 points, one operand above 2^15
    ]
    out = []
    for i in range(count):
        la, lb = kinds[int(g.integers(0, len(kinds)))]()
        lc = la + lb - 1
        assert lc <= 1 << 16
        out.append((primes[int(g.integers(0, 3))], la, lb))
    return out


@pytest.mark.parametrize("count", [3 * 256 + 1, 1100])
def test_mixed_class3_batch_more_items_than_workgroups(count, m15):
    torch_cuda()
    shapes = _mixed_shapes(count, 4100 + count)
    pairs, args = [], []
    for i, (p, la, lb) in enumerate(shapes):
        a = inputs.residues(p, la, inputs.CFG_TEST, 5000 + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 5000 + i, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        args.append((a, b, p))
    say("mixed class-3 batch of %d products, fused.m15.w32=%d" % (count, m15))
    got = ntt.polymul_batch(pairs, [s[0] for s in shapes])
    want = oracle_many(oracle.polymul_ntt, args)
    for i in range(count):
        assert_equal_u(ntt.to_numpy(got[i]), want[i], "mixed class-3 item %d %s" % (i, shapes[i]))
