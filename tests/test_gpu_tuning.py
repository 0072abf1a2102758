"""Every launch-shape choice the tuner may pick computes the same canonical result:
transforms and products under each row length, and single products on either side
of the fused-kernel threshold, against the oracle and against each other."""
import os

import numpy as np
import pytest

import oracle
from oracle import numtheory
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture()
def fresh():
    torch = torch_cuda()
    ntt.load()
    ntt.tune_clear()
    ntt.plan_cache_clear()
    yield torch
    torch.cuda.synchronize()
    ntt.tune_clear()
    if os.path.exists(ntt.TUNE_FILE):
        ntt.tune_load(ntt.TUNE_FILE)
    ntt.plan_cache_clear()


@pytest.mark.parametrize("p,L,cands", [(469762049, 18, (14, 13, 12)), (469762049, 15, (14, 13, 12)),
                                        (4611685941117976577, 16, (13, 12)), (4611685941117976577, 14, (13, 12))])
def test_transform_splits_agree(fresh, p, L, cands):
    torch = fresh
    x = inputs.residues(p, 1 << L, inputs.CFG_TEST, 1100 + L)
    dx = ntt.to_device(x)
    w = numtheory.root_of_unity(p, 1 << L)
    idx = np.array([0, 1, 7, 4097, (1 << L) - 1], dtype=np.int64)
    want = oracle.horner_many(x, p, np.array([pow(w, int(i), p) for i in idx], dtype=np.uint64))
    outs = []
    for c in cands:
        ntt.tune_set("split.w%d.L%d" % (ntt.word_bits(p), L), c)
        plan = ntt.Plan(p, L)
        assert plan.info.passes == 2 and plan.info.row_log2 == c
        say("transform p=%d L=%d rows 2^%d" % (p, L, c))
        y = plan.forward(dx)
        z = plan.inverse(y)
        torch.cuda.synchronize()
        yh = ntt.to_numpy(y)
        assert_equal_u(yh[idx], want, "forward values, rows 2^%d" % c)
        assert_equal_u(ntt.to_numpy(z), x, "round trip, rows 2^%d" % c)
        outs.append(yh)
        plan.close()
    for o in outs[1:]:
        assert_equal_u(o, outs[0], "forward across row lengths")


@pytest.mark.parametrize("p,la,lb,cands", [(998244353, 40000, 30001, (14, 13, 12)),
                                           (2013265921, 1 << 16, 1 << 16, (14, 13, 12)),
                                           (4611685941117976577, 20000, 15000, (13, 12))])
def test_product_splits_agree(fresh, p, la, lb, cands):
    a = inputs.residues(p, la, inputs.CFG_TEST, 1200, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 1200, 1)
    want = oracle.polymul_ntt(a, b, p, numtheory.smallest_generator(p))
    L = (la + lb - 2).bit_length()
    da, db = ntt.to_device(a), ntt.to_device(b)
    for c in cands:
        ntt.tune_set("psplit.w%d.L%d" % (ntt.word_bits(p), L), c)
        ntt.plan_cache_clear()
        say("product p=%d N=2^%d rows 2^%d" % (p, L, c))
        assert_equal_u(ntt.to_numpy(ntt.polymul(da, db, p)), want, "product, rows 2^%d" % c)


@pytest.mark.parametrize("p,n,limits", [(2013265921, 1 << 15, (14, 15, 16)), (998244353, 20000, (14, 15, 16)),
                                        (4611685941117976577, 1 << 14, (13, 14, 15))])
def test_single_product_fused_threshold(fresh, p, n, limits):
    a = inputs.residues(p, n, inputs.CFG_TEST, 1300, 0)
    b = inputs.residues(p, n, inputs.CFG_TEST, 1300, 1)
    want = oracle.polymul_ntt(a, b, p, numtheory.smallest_generator(p))
    da, db = ntt.to_device(a), ntt.to_device(b)
    for lim in limits:
        ntt.tune_set("fused.single.max.w%d" % ntt.word_bits(p), lim)
        say("single product p=%d n=%d fused up to 2^%d" % (p, n, lim))
        assert_equal_u(ntt.to_numpy(ntt.polymul(da, db, p)), want, "fused limit 2^%d" % lim)


@pytest.mark.parametrize("p,la,lb,L", [(998244353, 4096, 4096, 13), (998244353, 3000, 77, 12),
                                       (2013265921, 1 << 15, 1 << 15, 16), (2013265921, 1, 2047, 11),
                                       (469762049, 5000, 9000, 14), (4611685941117976577, 2048, 2048, 12),
                                       (4611685941117976577, 10000, 6000, 14)])
def test_single_product_split_paths(fresh, p, la, lb, L):
    a = inputs.residues(p, la, inputs.CFG_TEST, 1500 + L, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 1500 + L, 1)
    want = oracle.polymul_ntt(a, b, p, numtheory.smallest_generator(p))
    da, db = ntt.to_device(a), ntt.to_device(b)
    w = ntt.word_bits(p)
    for d in (1, 2, 3):
        if not 10 <= L - d <= (13 if w == 32 else 12):
            continue
        ntt.tune_set("single.split.w%d.L%d" % (w, L), d)
        say("split product p=%d la=%d lb=%d over 2^%d workgroups" % (p, la, lb, d))
        assert_equal_u(ntt.to_numpy(ntt.polymul(da, db, p)), want, "split depth %d" % d)


def test_intmul_under_fused_threshold_choices(fresh):
    a = inputs.limbs16(20000, inputs.CFG_TEST, 1400, 0)
    b = inputs.limbs16(12000, inputs.CFG_TEST, 1400, 1)
    want = oracle.intmul_pyint(a, b)
    for lim in (14, 16):
        ntt.tune_set("fused.single.max.w32", lim)
        got = ntt.to_numpy(ntt.intmul(ntt.to_device(a), ntt.to_device(b)))
        assert_equal_u(got, want, "intmul, fused limit 2^%d" % lim)


def test_autotuner_quick_run_writes_loadable_choices(fresh, tmp_path):
    from paper_1407_3383_amd import autotune
    out = tmp_path / "choices.txt"
    old = os.environ.get("NTT_TUNE_FILE")
    try:
        assert autotune.main(["--out", str(out), "--reps", "2", "--quick"]) == 0
    finally:
        if old is None:
            os.environ.pop("NTT_TUNE_FILE", None)
        else:
            os.environ["NTT_TUNE_FILE"] = old
    ntt.tune_clear()
    ntt.tune_load(str(out))
    keys = [ln.split()[0] for ln in open(out) if ln.split() and not ln.lstrip().startswith("#")]
    assert "fused.single.max.w32" in keys and "split.w32.L24" in keys
    assert all(ntt.tune_get(k) is not None for k in keys)


# TFT truncation: products whose lc leaves the top sub-problems without outputs
@pytest.mark.parametrize("p,la,lb,L,d", [
    (998244353, 20000, 20000, 16, 3), (998244353, 24000, 24000, 16, 3), (2013265921, 28000, 28000, 16, 3),
    (998244353, 9000, 9000, 15, 2), (469762049, 12000, 8000, 15, 2), (2013265921, 40000, 2, 16, 3),
    (4611685941117976577, 9000, 9000, 15, 3), (4611685941117976577, 5000, 4000, 14, 2)])
def test_split_truncated_products(fresh, p, la, lb, L, d):
    a = inputs.residues(p, la, inputs.CFG_TEST, 1600 + la, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 1600 + lb, 1)
    assert (la + lb - 2).bit_length() == L
    want = oracle.polymul_ntt(a, b, p, numtheory.smallest_generator(p))
    w = ntt.word_bits(p)
    ntt.tune_set("single.split.w%d.L%d" % (w, L), d)
    S = 1 << (L - d)
    say("split product p=%d la=%d lb=%d: %d of %d sub-problems" % (p, la, lb, -(-(la + lb - 1) // S), 1 << d))
    assert_equal_u(ntt.to_numpy(ntt.polymul(ntt.to_device(a), ntt.to_device(b), p)), want, "truncated split product")


def test_batch_fork_choices_agree(fresh):
    """A batch of every size class and of two-pass products, its launches forked onto
    streams of their own (the default) or all on the caller's stream: the same products,
    equal to the oracle's, through one-call batches and reusable handles."""
    torch = fresh
    primes = (998244353, 2013265921, 4611685941117976577)
    shapes = [(primes[i % 3], la, lb) for i, (la, lb) in enumerate(
        [(100, 29), (700, 300), (2000, 2049), (4000, 4000), (9000, 7000), (20000, 30000), (1 << 15, 1 << 15),
         (40000, 25000), (70000, 60000), (1 << 17, 5), (3, 1 << 18)])]
    pairs, args = [], []
    for i, (p, la, lb) in enumerate(shapes):
        a = inputs.residues(p, la, inputs.CFG_TEST, 1500 + i, 0)
        b = inputs.residues(p, lb, inputs.CFG_TEST, 1500 + i, 1)
        pairs.append((ntt.to_device(a), ntt.to_device(b)))
        args.append((a, b, p))
    want = [oracle.polymul_ntt(a, b, p) for a, b, p in args]
    for fork in (1, 0):
        ntt.tune_set("batch.fork", fork)
        say("batch of %d products, batch.fork=%d" % (len(shapes), fork))
        got = ntt.polymul_batch(pairs, [s[0] for s in shapes])
        outs = [torch.full_like(g, -1) for g in got]
        bt = ntt.Batch(pairs, [s[0] for s in shapes], outs)
        for _ in range(2):
            bt()
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert_equal_u(ntt.to_numpy(got[i]), want[i], "batch item %d, batch.fork=%d" % (i, fork))
            assert_equal_u(ntt.to_numpy(outs[i]), want[i], "handle item %d, batch.fork=%d" % (i, fork))
        bt.close()
