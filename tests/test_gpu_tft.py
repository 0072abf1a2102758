"""Truncated Fourier transforms (section 5.1) on the GPU against the oracle.

Forward: ntt_tft_forward's first l_out values in the TFT order, from l_in coefficients,
against the oracle's textbook transform of the zero-padded input reordered into the TFT
order (and, at small sizes, against the TFT definition by evaluation).  Inverse: from
the oracle's l TFT values the GPU must return the l coefficients exactly (the inverse
is unique), and at small sizes it must equal the oracle's inverse TFT by definition (a
linear solve).  One-pass plans (one LDS-resident vector) and two-pass plans (Algorithm 1
truncated at row granularity; l values that end inside a row take the column, row and
column inverse TFT steps), 32- and 64-bit words, batches with strides.  Products whose
two-pass transforms are truncated (the product's length between multiples of the row
length) are compared with the oracle's product."""
import numpy as np
import pytest

import oracle
from oracle import algorithm1 as alg
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, oracle_many, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)


def _plan(p, log2n):
    pl = ntt.Plan(p, log2n)
    return pl, nt.root_of_unity(p, 1 << log2n, pl.info.g)


def _lengths(n, n1, seed):
    g = inputs.rng(inputs.CFG_TEST, seed)
    ls = {1, 2, n, n - 1, n // 2, n // 2 + 1, n1, n1 + 1, max(1, n1 - 1), min(n, 3 * n1 + 17)}
    ls |= {int(g.integers(1, n + 1)) for _ in range(4)}
    return sorted(x for x in ls if 1 <= x <= n)


@pytest.mark.parametrize("p,log2n", [(998244353, 4), (998244353, 10), (2013265921, 13), (469762049, 14),
                                     (P62, 9), (P62, 13),
                                     (998244353, 15), (2013265921, 16), (469762049, 18), (998244353, 20),
                                     (P62, 15), (P62, 17)])
def test_tft_forward_and_inverse(p, log2n):
    torch = torch_cuda()
    pl, w = _plan(p, log2n)
    n = 1 << log2n
    n1 = 1 << pl.info.row_log2 if pl.info.passes > 1 else n
    for l in _lengths(n, n1, log2n * 7 + p % 97):
        a = inputs.residues(p, l, inputs.CFG_TEST, 12000 + l % 1000, log2n)
        want = oracle.tft(a, n, l, p, w)
        say("tft p=%d n=2^%d l=%d (rows of %d)" % (p, log2n, l, n1))
        got = ntt.to_numpy(pl.tft(ntt.to_device(a), l))
        assert_equal_u(got, want, "tft forward p=%d n=2^%d l=%d" % (p, log2n, l))
        back = ntt.to_numpy(pl.itft(ntt.to_device(want.astype(a.dtype)), l))
        assert_equal_u(back, a, "tft inverse p=%d n=2^%d l=%d" % (p, log2n, l))
    torch.cuda.synchronize()
    pl.close()


@pytest.mark.parametrize("p,log2n", [(998244353, 5), (2013265921, 6), (P62, 6)])
def test_tft_small_against_definitions(p, log2n):
    torch_cuda()
    pl, w = _plan(p, log2n)
    n = 1 << log2n
    for l in range(1, n + 1, 3):
        a = inputs.residues(p, l, inputs.CFG_TEST, 12500 + l, log2n)
        got = [int(x) for x in ntt.to_numpy(pl.tft(ntt.to_device(a), l))]
        assert got == alg.tft_definition([int(x) for x in a], l, n, w, p), (p, log2n, l)
        vals = inputs.residues(p, l, inputs.CFG_TEST, 12600 + l, log2n)  # arbitrary TFT values
        inv = [int(x) for x in ntt.to_numpy(pl.itft(ntt.to_device(vals), l))]
        assert inv == alg.itft_definition([int(x) for x in vals], l, n, w, p), (p, log2n, l)
    pl.close()


@pytest.mark.parametrize("p,log2n,l_in,l_out", [(998244353, 12, 100, 4000), (998244353, 18, 70000, 100000),
                                                (2013265921, 17, 131072, 5000), (P62, 16, 3, 65536),
                                                (469762049, 16, 0, 777), (469762049, 16, 9000, 0)])
def test_tft_forward_lengths_differ(p, log2n, l_in, l_out):
    torch_cuda()
    pl, w = _plan(p, log2n)
    n = 1 << log2n
    a = inputs.residues(p, l_in, inputs.CFG_TEST, 12700, log2n)
    say("tft p=%d n=2^%d l_in=%d l_out=%d" % (p, log2n, l_in, l_out))
    x = ntt.to_device(a) if l_in else ntt.to_device(np.zeros(1, dtype=a.dtype))
    got = ntt.to_numpy(pl.tft(x, l_out, l_in=l_in))[:l_out]
    assert_equal_u(got, oracle.tft(a, n, l_out, p, w), "tft p=%d l_in=%d l_out=%d" % (p, l_in, l_out))
    pl.close()


@pytest.mark.parametrize("p,log2n,l", [(998244353, 11, 1500), (998244353, 19, 300000), (P62, 16, 40000)])
def test_tft_batches_with_strides(p, log2n, l):
    torch = torch_cuda()
    pl, w = _plan(p, log2n)
    n = 1 << log2n
    batch, stride = 3, l + 37
    A = [inputs.residues(p, l, inputs.CFG_TEST, 12800 + b, log2n) for b in range(batch)]
    flat = np.zeros(batch * stride, dtype=A[0].dtype)
    for b in range(batch):
        flat[b * stride:b * stride + l] = A[b]
    say("tft batch p=%d n=2^%d l=%d" % (p, log2n, l))
    dX = ntt.to_device(flat)
    T = pl.tft(dX, l, l_in=l, batch=batch, in_stride=stride, out_stride=stride)
    Tn = ntt.to_numpy(T)
    wants = oracle_many(lambda x: oracle.tft(x, n, l, p, w), [(A[b],) for b in range(batch)])
    for b in range(batch):
        assert_equal_u(Tn[b * stride:b * stride + l], wants[b], "tft batch item %d" % b)
    back = ntt.to_numpy(pl.itft(T, l, batch=batch, in_stride=stride, out_stride=stride))
    for b in range(batch):
        assert_equal_u(back[b * stride:b * stride + l], A[b], "itft batch item %d" % b)
    torch.cuda.synchronize()
    pl.close()


@pytest.mark.parametrize("p", [998244353, 2013265921, P62])
@pytest.mark.parametrize("la,lb", [(40000, 30000), (65536, 1), (4097, 61440), (100001, 100000), (70000, 62000),
                                   ((1 << 17) + 5, 9000), (300000, 200001)])
def test_products_with_truncated_two_pass_transforms(p, la, lb):
    torch_cuda()
    a = inputs.residues(p, la, inputs.CFG_TEST, 12900 + la % 997, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 12900 + lb % 997, 1)
    want = oracle.polymul_ntt(a, b, p)
    key = "tft.rows.w%d" % ntt.word_bits(p)
    for mode in (1, 0):  # truncated at row granularity, then full length (the default)
        ntt.tune_set(key, mode)
        say("product p=%d la=%d lb=%d tft.rows=%d" % (p, la, lb, mode))
        try:
            c = ntt.to_numpy(ntt.polymul(ntt.to_device(a), ntt.to_device(b), p))
        finally:
            ntt.tune_set(key, 0)
        assert_equal_u(c, want, "product p=%d la=%d lb=%d tft.rows=%d" % (p, la, lb, mode))


def test_tft_argument_errors():
    torch = torch_cuda()
    pl, _ = _plan(998244353, 12)
    x = torch.zeros(8192, dtype=torch.int32, device="cuda")
    with pytest.raises(ntt.NTTError) as e:
        pl.tft(x, 5000, l_in=5000)  # l_out > n
    assert e.value.code == ntt.NTT_EINVAL
    with pytest.raises(ntt.NTTError) as e:
        pl.itft(x, 4097)
    assert e.value.code == ntt.NTT_EINVAL
    pl.close()
