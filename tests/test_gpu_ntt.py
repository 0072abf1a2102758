"""GPU parity of the transforms (section 5.1) against the CPU oracle, bit-exact."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)
GENS = {998244353: 3, 2013265921: 31, 469762049: 3, 167772161: 3, P62: None}


def _plan(p, log2n, flags=0):
    g = GENS.get(p) or nt.smallest_generator(p)
    return ntt.Plan(p, log2n, g, flags), nt.root_of_unity(p, 1 << log2n, g)


@pytest.mark.parametrize("p", [998244353, 2013265921, 469762049, P62])
@pytest.mark.parametrize("log2n", [0, 1, 2, 3, 4, 5, 7, 10, 11, 12, 13, 14, 15, 16, 18])
@pytest.mark.parametrize("bitrev", [False, True])
def test_forward_inverse_exact(p, log2n, bitrev):
    torch_cuda()
    n = 1 << log2n
    batch = 3 if log2n <= 14 else 1
    flags = (ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN) if bitrev else 0
    plan, w = _plan(p, log2n, flags)
    x = np.stack([inputs.residues(p, n, inputs.CFG_TEST, 50 + log2n, i) for i in range(batch)])
    say("ntt p=%d log2n=%d bitrev=%s batch=%d passes=%d" % (p, log2n, bitrev, batch, plan.info.passes))
    X = plan.forward(ntt.to_device(x.reshape(-1)), batch=batch)
    got = ntt.to_numpy(X).reshape(batch, n)
    for i in range(batch):
        ref = oracle.ntt(x[i], p, w)
        if bitrev:
            ref = oracle.tft_order(ref)
        assert_equal_u(got[i], ref, "forward vec %d" % i)
    back = ntt.to_numpy(plan.inverse(X, batch=batch)).reshape(batch, n)
    assert_equal_u(back.reshape(-1), x.reshape(-1), "inverse(forward)")


@pytest.mark.parametrize("p,log2n", [(469762049, 20), (998244353, 22), (2013265921, 21), (P62, 19), (P62, 21)])
def test_large_transform_exact(p, log2n):
    """Two-pass transforms compared element by element with the oracle's textbook
    transform (TFT order), plus evaluations at random points as a check independent of
    the oracle's transform, and the round trip."""
    torch_cuda()
    n = 1 << log2n
    plan, w = _plan(p, log2n, ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN)
    x = inputs.residues(p, n, inputs.CFG_TEST, 70 + log2n)
    say("ntt large p=%d log2n=%d passes=%d" % (p, log2n, plan.info.passes))
    X = plan.forward(ntt.to_device(x))
    Xh = ntt.to_numpy(X)
    assert_equal_u(Xh, oracle.tft_order(oracle.ntt(x, p, w)), "forward vs oracle transform")
    rng = np.random.default_rng(log2n)
    idx = rng.integers(0, n, size=16)
    pts = [pow(w, oracle.bitrev(int(i), log2n), p) for i in idx]
    assert_equal_u(Xh[idx], oracle.horner_many(x, p, pts), "forward spot checks")
    assert_equal_u(ntt.to_numpy(plan.inverse(X)), x, "roundtrip")


def test_ntt_2_24_exact():
    torch_cuda()
    p, x = inputs.ntt_2_24_inputs()
    plan, w = _plan(p, 24, ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN)
    say("ntt 2^24 p=%d passes=%d" % (p, plan.info.passes))
    X = plan.forward(ntt.to_device(x))
    Xh = ntt.to_numpy(X)
    assert_equal_u(Xh, oracle.tft_order(oracle.ntt(x, p, w)), "2^24 forward vs oracle transform")
    rng = np.random.default_rng(24)
    idx = rng.integers(0, 1 << 24, size=16)
    pts = [pow(w, oracle.bitrev(int(i), 24), p) for i in idx]
    assert_equal_u(Xh[idx], oracle.horner_many(x, p, pts), "2^24 forward spot checks")
    assert_equal_u(ntt.to_numpy(plan.inverse(X)), x, "2^24 roundtrip")


def test_ntt_2_24_natural_order_exact():
    torch_cuda()
    p, x = inputs.ntt_2_24_inputs()
    plan, w = _plan(p, 24, 0)
    X = plan.forward(ntt.to_device(x))
    Xh = ntt.to_numpy(X)
    assert_equal_u(Xh, oracle.ntt(x, p, w), "2^24 natural-order forward vs oracle transform")
    assert_equal_u(ntt.to_numpy(plan.inverse(X)), x, "natural roundtrip")


def test_validate_flag_rejects_noncanonical():
    torch_cuda()
    p = 998244353
    plan = ntt.Plan(p, 10, 3, ntt.NTT_VALIDATE)
    x = inputs.residues(p, 1024, inputs.CFG_TEST, 1)
    x[17] = p
    with pytest.raises(ntt.NTTError) as e:
        plan.forward(ntt.to_device(x))
    assert e.value.code == ntt.NTT_ERANGE
    x[17] = p - 1
    plan.forward(ntt.to_device(x))


@pytest.mark.parametrize("p,log2n", [(469762049, 26), (2013265921, 25), (P62, 24)])
def test_maximum_length_transforms(p, log2n):
    """The longest transforms the plans take (2^26 words; the column pass then runs its
    rounds across workgroups): evaluations at random points of the TFT-order output,
    the first and last values, and the round trip."""
    torch_cuda()
    n = 1 << log2n
    plan, w = _plan(p, log2n, ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN)
    x = inputs.residues(p, n, inputs.CFG_TEST, 90 + log2n)
    say("ntt maximum p=%d log2n=%d passes=%d" % (p, log2n, plan.info.passes))
    X = plan.forward(ntt.to_device(x))
    Xh = ntt.to_numpy(X)
    rng = np.random.default_rng(log2n + 1)
    idx = np.concatenate([[0, 1, n - 1], rng.integers(0, n, size=8)])
    pts = [pow(w, oracle.bitrev(int(i), log2n), p) for i in idx]
    assert_equal_u(Xh[idx], oracle.horner_many(x, p, pts), "maximum-length forward at sampled points")
    assert_equal_u(ntt.to_numpy(plan.inverse(X)), x, "maximum-length roundtrip")
