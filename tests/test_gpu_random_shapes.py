"""Seeded random shapes against the oracle: batches that mix primes, size classes and
ragged lengths (every fused class, the TFT boundaries, the two-pass path), products
with residues in doubles, and integer products of random sizes (16-bit limbs and
32-bit chunks).  Each case prints its seed and shapes before it runs."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)
P49 = nt.largest_prime_below(49, 20)
PRIMES = [998244353, 2013265921, 469762049, 7340033, P62]


def _lengths(g, n, lo_log2, hi_log2):
    return [max(1, int(2 ** g.uniform(lo_log2, hi_log2))) for _ in range(n)]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_mixed_batches(seed):
    torch_cuda()
    g = np.random.default_rng(31000 + seed)
    las, lbs = _lengths(g, 24, 0, 16.2), _lengths(g, 24, 0, 16.2)
    ps = [PRIMES[int(g.integers(len(PRIMES)))] for _ in range(24)]
    pairs, want, specs = [], [], []
    for i, (la, lb, p) in enumerate(zip(las, lbs, ps)):
        if p == P62:  # 64-bit words: keep the oracle's transform product quick
            la, lb = min(la, 40000), min(lb, 40000)
        a = inputs.residues(p, la, inputs.CFG_TEST, 31000 + 100 * seed + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 31000 + 100 * seed + i, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        want.append(oracle.polymul_ntt(a, b, p))
        specs.append((p, la, lb))
    say("random batch seed %d: %s" % (seed, specs))
    outs = ntt.polymul_batch(pairs, ps)
    for i, (o, w) in enumerate(zip(outs, want)):
        assert_equal_u(ntt.to_numpy(o), w, "seed %d item %d %s" % (seed, i, specs[i]))
    # the same products one call each (single-product paths: fused, split, two-pass)
    for i, ((da, db), p) in enumerate(zip(pairs[:8], ps[:8])):
        assert_equal_u(ntt.to_numpy(ntt.polymul(da, db, p)), want[i], "seed %d single %d %s" % (seed, i, specs[i]))


@pytest.mark.parametrize("seed", [1, 2])
def test_random_f64_batches(seed):
    torch = torch_cuda()
    g = np.random.default_rng(32000 + seed)
    specs = []
    for _ in range(12):
        la, lb = _lengths(g, 1, 0, 14)[0], _lengths(g, 1, 0, 14)[0]
        p = [998244353, nt.largest_prime_below(48, 20), P49][int(g.integers(3))]
        specs.append((p, la, lb))
    say("random f64 batch seed %d: %s" % (seed, specs))
    pairs, outs, want = [], [], []
    for i, (p, la, lb) in enumerate(specs):
        a = inputs.residues(p, la, inputs.CFG_TEST, 32000 + 100 * seed + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 32000 + 100 * seed + i, 1)
        pairs.append((torch.from_numpy(a.astype(np.float64)).cuda(), torch.from_numpy(b.astype(np.float64)).cuda()))
        outs.append(torch.empty(la + lb - 1, dtype=torch.float64, device="cuda"))
        want.append(oracle.polymul_ntt(a, b, p))
    descs = (ntt.PolymulDesc * len(specs))()
    for i, ((a, b), c, (p, la, lb)) in enumerate(zip(pairs, outs, specs)):
        descs[i] = ntt.PolymulDesc(p, a.data_ptr(), la, b.data_ptr(), lb, c.data_ptr())
    L = ntt.load()
    ws = torch.empty(max(L.polymul_f64_batch_workspace_bytes(descs, len(specs)), 1), dtype=torch.uint8, device="cuda")
    ntt._check(L.polymul_f64_batch(descs, len(specs), ntt._ptr(ws), ws.numel(), None), "polymul_f64_batch")
    torch.cuda.synchronize()
    for i, (c, w) in enumerate(zip(outs, want)):
        assert_equal_u(c.cpu().numpy().astype(np.uint64), w, "f64 seed %d item %d %s" % (seed, i, specs[i]))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_integer_products(seed):
    torch_cuda()
    g = np.random.default_rng(33000 + seed)
    for k in range(4):
        na, nb = _lengths(g, 1, 0, 18)[0], _lengths(g, 1, 0, 18)[0]
        a = inputs.limbs16(na, inputs.CFG_TEST, 33000 + 10 * seed + k, 0)
        b = inputs.limbs16(nb, inputs.CFG_TEST, 33000 + 10 * seed + k, 1)
        say("random intmul seed %d: %d x %d limbs" % (seed, na, nb))
        got = ntt.to_numpy(ntt.intmul(ntt.to_device(a), ntt.to_device(b)))
        assert_equal_u(got, oracle.intmul_pyint(a, b), "intmul seed %d %dx%d" % (seed, na, nb))
        ma, mb = max(1, na // 2), max(1, nb // 2)
        a32 = inputs.limbs32(ma, inputs.CFG_TEST, 33500 + 10 * seed + k, 0)
        b32 = inputs.limbs32(mb, inputs.CFG_TEST, 33500 + 10 * seed + k, 1)
        got32 = ntt.to_numpy(ntt.intmul32(ntt.to_device(a32), ntt.to_device(b32)))
        A = int.from_bytes(a32.astype("<u4").tobytes(), "little")
        B = int.from_bytes(b32.astype("<u4").tobytes(), "little")
        want32 = np.frombuffer((A * B).to_bytes(4 * (ma + mb), "little"), dtype="<u4")
        assert_equal_u(got32, want32, "intmul32 seed %d %dx%d" % (seed, ma, mb))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_matrix_products(seed):
    torch = torch_cuda()
    g = np.random.default_rng(34000 + seed)
    for k in range(3):
        n = int(g.integers(1, 65))
        d = max(1, int(2 ** g.uniform(0, 7 if n > 16 else 10)))
        p = [469762049, 998244353, 2013265921, 7340033][int(g.integers(4))]
        A = inputs.residues(p, n * n * d, inputs.CFG_TEST, 34000 + 10 * seed + k, 0).reshape(n, n, d)
        B = inputs.residues(p, n * n * d, inputs.CFG_TEST, 34000 + 10 * seed + k, 1).reshape(n, n, d)
        say("random polymatmul seed %d: p=%d n=%d d=%d" % (seed, p, n, d))
        C = ntt.polymatmul(ntt.to_device(A.reshape(-1)).reshape(n, n, d), ntt.to_device(B.reshape(-1)).reshape(n, n, d), p)
        torch.cuda.synchronize()
        assert_equal_u(ntt.to_numpy(C.reshape(-1)), oracle.polymatmul(A, B, p).reshape(-1),
                       "polymatmul seed %d p=%d n=%d d=%d" % (seed, p, n, d))
    n = int(g.integers(1, 13))
    na = max(1, int(2 ** g.uniform(0, 9)))
    A = inputs.limbs32(n * n * na, inputs.CFG_TEST, 34500 + seed, 0).reshape(n, n, na)
    B = inputs.limbs32(n * n * na, inputs.CFG_TEST, 34500 + seed, 1).reshape(n, n, na)
    say("random intmatmul seed %d: n=%d na=%d" % (seed, n, na))
    C = ntt.intmatmul32(ntt.to_device(A.reshape(-1)).reshape(n, n, na), ntt.to_device(B.reshape(-1)).reshape(n, n, na))
    torch.cuda.synchronize()
    assert_equal_u(ntt.to_numpy(C.reshape(-1)).astype(np.uint32), oracle.intmatmul_pyint(A, B).reshape(-1),
                   "intmatmul seed %d n=%d na=%d" % (seed, n, na))
