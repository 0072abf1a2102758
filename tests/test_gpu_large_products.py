"""Products at the serving mix's largest sizes (operands up to 2^20 coefficients, so
transform lengths up to 2^21), which take the two-pass path of Algorithm 1 with the
fused row product, against the oracle bit-exactly: for 998244353, 2013265921 and the
~62-bit prime.  And the native serving loop on a mix whose lengths are drawn
log-uniformly from [2^15, 2^20], every result against the oracle."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt, serve

from gpu_util import assert_equal_u, oracle_many, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)


@pytest.mark.parametrize("p", [998244353, 2013265921, P62])
@pytest.mark.parametrize("la,lb", [(1 << 17, 1 << 17), ((1 << 18) + 123, (1 << 18) + 123), (1 << 19, 1 << 19),
                                   (1 << 20, 1 << 20), ((1 << 20) - 5, 77777)])
def test_polymul_serving_sizes(p, la, lb):
    torch_cuda()
    a = inputs.residues(p, la, inputs.CFG_TEST, 9000 + la % 1000, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 9000 + lb % 1000, 1)
    say("polymul p=%d la=%d lb=%d" % (p, la, lb))
    c = ntt.to_numpy(ntt.polymul(ntt.to_device(a), ntt.to_device(b), p))
    assert_equal_u(c, oracle.polymul_ntt(a, b, p), "polymul p=%d la=%d lb=%d" % (p, la, lb))


def test_native_server_large_requests():
    torch_cuda()
    primes = (998244353, 2013265921, P62)
    specs = inputs.serve_requests(24, primes, 15.0, 20.0, 11)
    arrivals = inputs.poisson_arrivals(24, 2000.0, 11)
    reqs = []
    for (p, L, rid), t in zip(specs, arrivals):
        a, b = inputs.serve_operands(p, L, rid)
        reqs.append(serve.Request(rid, p, a, b, arrival=float(t)))
    say("native server: %d requests with L in [2^15, 2^20]" % len(reqs))
    srv = serve.NativeServer(budget_bytes=1 << 30, streams=4, max_batch=16)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    st = srv.stats()
    assert st["pending"] == 0 and st["inflight"] == 0 and st["arena_used"] == 0
    want = oracle_many(oracle.polymul_ntt, [(r.a, r.b, r.p) for r in reqs])
    for r, w in zip(reqs, want):
        assert_equal_u(r.result, w, "native request %d (p=%d, L=%d) vs oracle" % (r.rid, r.p, r.a.size))
    srv.close()


@pytest.mark.parametrize("p,la,lb", [(469762049, 1 << 25, (1 << 25) + 1 - 1), (469762049, (1 << 26) - 5, 6),
                                     (nt.largest_prime_below(62, 32), 1 << 23, (1 << 23) - 1)])
def test_products_at_maximum_length(p, la, lb):
    """Products whose transform is the longest a plan takes (2^26 words for 32-bit
    primes): c(x) = a(x) b(x) at random points x (an identity at any size, independent
    of any transform), and the lowest and highest coefficients."""
    torch_cuda()
    a = inputs.residues(p, la, inputs.CFG_TEST, 9100, 0)
    b = inputs.residues(p, lb, inputs.CFG_TEST, 9100, 1)
    say("maximum-length product p=%d la=%d lb=%d" % (p, la, lb))
    c = ntt.to_numpy(ntt.polymul(ntt.to_device(a), ntt.to_device(b), p))
    assert c.size == la + lb - 1
    xs = [int(v) for v in inputs.residues(p, 6, inputs.CFG_TEST, 9101, 0)]
    ea, eb, ec = oracle.horner_many(a, p, xs), oracle.horner_many(b, p, xs), oracle.horner_many(c, p, xs)
    for k in range(len(xs)):
        assert int(ec[k]) == int(ea[k]) * int(eb[k]) % p, "product at x = %d" % xs[k]
    assert int(c[0]) == int(a[0]) * int(b[0]) % p
    assert int(c[-1]) == int(a[-1]) * int(b[-1]) % p
