"""Serving loop (continuous batching by HBM budget): every result is the same when
the request is served alone and in the mix, bit-exact, and matches the oracle."""
import numpy as np
import pytest

import oracle
from oracle import numtheory as nt
from paper_1407_3383_amd import inputs, ntt, serve

from gpu_util import assert_equal_u, say, torch_cuda

pytestmark = pytest.mark.gpu

P62 = nt.largest_prime_below(62, 32)
PRIMES = (998244353, 2013265921, P62)


def _requests(n, rate, lo=8.0, hi=14.0, seed=0):
    specs = inputs.serve_requests(n, PRIMES, lo, hi, seed)
    arrivals = inputs.poisson_arrivals(n, rate, seed)
    out = []
    for (p, L, rid), t in zip(specs, arrivals):
        a, b = inputs.serve_operands(p, L, rid)
        out.append(serve.Request(rid, p, a, b, arrival=float(t)))
    return out


def _alone(r):
    c = ntt.polymul(ntt.to_device(r.a), ntt.to_device(r.b), r.p)
    return ntt.to_numpy(c)


def test_serve_mix_equals_alone_and_oracle():
    torch_cuda()
    reqs = _requests(60, rate=20000.0)
    say("serve mix of %d requests" % len(reqs))
    srv = serve.Server(budget_bytes=256 << 20, streams=4, max_batch=16)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    assert srv.max_inflight_batches >= 2, "no batches overlapped on the device"
    for r in reqs:
        assert_equal_u(r.result, _alone(r), "request %d (p=%d, L=%d) mix vs alone" % (r.rid, r.p, r.a.size))
    for r in reqs[:12]:
        assert_equal_u(r.result, oracle.polymul_ntt(r.a, r.b, r.p), "request %d vs oracle" % r.rid)
    stats = serve.latency_stats(srv.completed)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_serve_small_budget_queues_and_completes():
    torch_cuda()
    reqs = _requests(24, rate=1e6, lo=10.0, hi=13.0, seed=1)
    biggest = max(serve.footprint(r.p, r.a.size, r.b.size) for r in reqs)
    srv = serve.Server(budget_bytes=biggest + (64 << 10), streams=2, max_batch=8)
    say("serve with a budget of %d bytes" % srv.arena.budget)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    for r in reqs:
        assert_equal_u(r.result, _alone(r), "request %d under a small budget" % r.rid)
    assert srv.arena.used == 0


def test_serve_admits_while_batches_in_flight():
    torch_cuda()
    reqs = _requests(80, rate=50000.0, lo=12.0, hi=16.0, seed=2)
    srv = serve.Server(budget_bytes=512 << 20, streams=4, max_batch=8)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    assert srv.overlapped_admissions > 0
    for r in reqs[::7]:
        assert_equal_u(r.result, _alone(r), "request %d" % r.rid)


def test_serve_rejects_request_beyond_budget():
    torch_cuda()
    reqs = _requests(2, rate=1000.0, lo=14.0, hi=14.5, seed=3)
    srv = serve.Server(budget_bytes=4096)
    with pytest.raises(ValueError):
        srv.run(reqs)


def test_serve_mixes_integer_and_polynomial_requests():
    torch_cuda()
    polys = _requests(30, rate=20000.0, lo=8.0, hi=14.0, seed=3)
    g = np.random.default_rng(np.random.SeedSequence([14073383, 7, 3]))
    ints = []
    for k in range(12):
        na = int(2 ** g.uniform(4, 15))
        nb = int(2 ** g.uniform(4, 15))
        a = inputs.limbs16(na, inputs.CFG_SERVE, 5000 + k, 0)
        b = inputs.limbs16(nb, inputs.CFG_SERVE, 5000 + k, 1)
        ints.append(serve.Request(90000 + k, 0, a, b, arrival=float(polys[2 * k].arrival), kind="int"))
    reqs = polys + ints
    say("serve mix of %d polynomial and %d integer products" % (len(polys), len(ints)))
    srv = serve.Server(budget_bytes=256 << 20, streams=4, max_batch=16)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    for r in ints:
        alone = ntt.to_numpy(ntt.intmul(ntt.to_device(r.a), ntt.to_device(r.b)))
        assert_equal_u(r.result, alone, "integer request %d mix vs alone" % r.rid)
        assert_equal_u(r.result, oracle.intmul_pyint(r.a, r.b), "integer request %d vs Python int" % r.rid)
    for r in polys:
        assert_equal_u(r.result, _alone(r), "request %d mix vs alone" % r.rid)
    assert srv.arena.used == 0


# ---------------------------------------------------------------- native request loop

def test_native_server_mix_equals_alone_and_oracle():
    torch_cuda()
    polys = _requests(50, rate=30000.0, lo=8.0, hi=15.0, seed=5)
    ints = []
    for k in range(8):
        n = 200 + 3000 * k
        a = inputs.limbs16(n, inputs.CFG_SERVE, 7000 + k, 0)
        b = inputs.limbs16(n // 2 + 1, inputs.CFG_SERVE, 7000 + k, 1)
        ints.append(serve.Request(80000 + k, 0, a, b, arrival=float(polys[3 * k].arrival), kind="int"))
    reqs = polys + ints
    srv = serve.NativeServer(budget_bytes=256 << 20, streams=4, max_batch=16)
    say("native server: %d polynomial and %d integer products" % (len(polys), len(ints)))
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    st = srv.stats()
    assert st["pending"] == 0 and st["inflight"] == 0 and st["arena_used"] == 0
    assert st["max_inflight"] >= 2, "no batches overlapped on the device"
    for r in polys:
        assert_equal_u(r.result, _alone(r), "native request %d mix vs alone" % r.rid)
    for r in polys[:10]:
        assert_equal_u(r.result, oracle.polymul_ntt(r.a, r.b, r.p), "native request %d vs oracle" % r.rid)
    for r in ints:
        assert_equal_u(r.result, oracle.intmul_pyint(r.a, r.b), "native integer request %d vs Python int" % r.rid)
    srv.close()


def test_native_server_small_budget_and_refusal():
    torch_cuda()
    reqs = _requests(20, rate=1e6, lo=10.0, hi=13.0, seed=6)
    biggest = max(serve.footprint(r.p, r.a.size, r.b.size) for r in reqs)
    srv = serve.NativeServer(budget_bytes=biggest + (1 << 20), streams=2, max_batch=8)
    srv.run(reqs)
    assert len(srv.completed) == len(reqs)
    for r in reqs:
        assert_equal_u(r.result, _alone(r), "native request %d under a small budget" % r.rid)
    srv.close()
    tiny = serve.NativeServer(budget_bytes=4096)
    with pytest.raises(ValueError):
        tiny.run(_requests(2, rate=1000.0, lo=14.0, hi=14.5, seed=7))
    tiny.close()


def test_native_server_without_copy_back():
    """Requests whose products stay on the device (c = NULL): every request completes
    and the server ends empty."""
    torch_cuda()
    reqs = _requests(60, rate=1e6, lo=8.0, hi=14.0, seed=8)
    srv = serve.NativeServer(budget_bytes=128 << 20, streams=4, max_batch=16, keep_results=False)
    srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in srv.completed) == sorted(r.rid for r in reqs)
    assert all(r.result is None for r in srv.completed)
    st = srv.stats()
    assert st["pending"] == 0 and st["inflight"] == 0 and st["arena_used"] == 0
    srv.close()


def test_native_server_pinned_results():
    """Results in page-locked host memory are filled by DMA directly (no staging copy):
    the same values as the request served alone and as the oracle."""
    torch_cuda()
    polys = _requests(40, rate=1e6, lo=8.0, hi=15.0, seed=9)
    ints = []
    for k in range(4):
        n = 300 + 2000 * k
        a = inputs.limbs16(n, inputs.CFG_SERVE, 7100 + k, 0)
        b = inputs.limbs16(n // 3 + 1, inputs.CFG_SERVE, 7100 + k, 1)
        ints.append(serve.Request(81000 + k, 0, a, b, arrival=0.0, kind="int"))
    srv = serve.NativeServer(budget_bytes=256 << 20, streams=4, max_batch=16, pinned_results=True)
    srv.run(polys + ints, realtime=False)
    assert len(srv.completed) == len(polys) + len(ints)
    for r in polys:
        assert_equal_u(r.result, _alone(r), "pinned native request %d mix vs alone" % r.rid)
    for r in polys[:6]:
        assert_equal_u(r.result, oracle.polymul_ntt(r.a, r.b, r.p), "pinned native request %d vs oracle" % r.rid)
    for r in ints:
        assert_equal_u(r.result, oracle.intmul_pyint(r.a, r.b), "pinned integer request %d vs Python int" % r.rid)
    srv.close()


def test_native_server_serves_again_into_the_same_buffers():
    """A second run of the same requests writes into the host buffers of the first (the
    caller's buffers, reused), with the products the requests have alone; with no copy
    threads the staging copies run on the driving thread."""
    torch_cuda()
    reqs = _requests(40, rate=1e6, lo=8.0, hi=16.0, seed=12)
    for threads in (7, 0):
        ntt.tune_set("server.copy_threads", threads)
        try:
            srv = serve.NativeServer(budget_bytes=256 << 20, streams=4, max_batch=16)
            srv.run(reqs, realtime=False)
            srv.close()
            bufs = [r.result for r in reqs]
            for b in bufs:
                b.fill(7)
            say("native server again into the same buffers, %d copy threads" % threads)
            srv = serve.NativeServer(budget_bytes=256 << 20, streams=4, max_batch=16)
            srv.run(reqs, realtime=False)
            st = srv.stats()
            srv.close()
        finally:
            ntt.tune_set("server.copy_threads", 7)
        assert st["pending"] == 0 and st["inflight"] == 0 and st["arena_used"] == 0
        for r, b in zip(reqs, bufs):
            assert r.result is b
            assert_equal_u(r.result, _alone(r), "request %d served again (%d copy threads)" % (r.rid, threads))
