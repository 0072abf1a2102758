"""Secondary benchmark workloads (bench.py --workload ...): one product of two
length-4096 operands mod 998244353, a length-2^24 forward + inverse transform mod
469762049, and the 2^21 x 2^21-limb three-prime integer product.  Each prints one
JSON line with the same keys as the headline line; inputs are resident in HBM and
plan creation is outside the timed region."""
from __future__ import annotations

import sys
import time

# Integer-VALU issue: 256 CUs x 64 lanes x 2.4 GHz full-rate lane-operation slots per
# second (32-bit multiplies, multiply-adds and min take one slot, plain add and subtract
# half of one: measured, paper_1407_3383_amd.valu_rates).  A butterfly of a prime below
# 2^30 (lazy ranges) takes 6 slots, one of a 31-bit prime 7.5; a multiply-add of the
# matrix products one.
ALU_SLOTS_PER_S = 256 * 64 * 2.4e9
SLOTS_PER_BFLY = 6.0
HBM_PEAK_GBPS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _time(fn, stream, steps, warmup):
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:  # untimed: let the GPU clocks ramp up
        for _ in range(max(warmup, 4)):
            fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    return wall_ms, e0.elapsed_time(e1) / steps


def _alu(slots, ms):
    """Integer-VALU roofline of a step that needs `slots` full-rate issue slots."""
    achieved = slots / (ms * 1e-3) / 1e12
    peak = ALU_SLOTS_PER_S / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "T issue slots/s (full-rate 32-bit VALU lane-operations; %.1f per butterfly)" % SLOTS_PER_BFLY,
            "frac": round(achieved / peak, 4)}


def _hbm(nbytes, ms):
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"algorithmic_bytes_per_step": int(nbytes), "achieved_GBps": round(gbps, 1),
            "frac": round(gbps / HBM_PEAK_GBPS, 4)}


def _line(metric, value, unit, ms, steps, warmup, config, extra):
    out = {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic", "config": config}
    out.update(extra)
    return out


def run(name, args):
    import numpy as np
    import torch

    from paper_1407_3383_amd import inputs, ntt
    stream = torch.cuda.Stream()
    if name == "polymul8k":
        p, a, b = inputs.polymul_8k_inputs()
        da, db = ntt.to_device(a), ntt.to_device(b)
        dc = torch.empty(8191, dtype=torch.int32, device="cuda")
        L = ntt.load()
        ws = torch.empty(max(L.polymul_workspace_bytes(p, 4096, 4096), 1), dtype=torch.uint8, device="cuda")
        split = ntt.tune_get("single.split.w32.L13") or 0

        def step():
            ntt._check(L.polymul_modp(p, ntt._ptr(da), 4096, ntt._ptr(db), 4096, ntt._ptr(dc), ntt._ptr(ws),
                                      ws.numel(), ntt._stream(stream)), "polymul_modp")
        steps = max(args.steps, 200)
        ms, kms = _time(step, stream, steps, 20)
        # device time per product without the host's call overhead: 100 calls in one graph
        g = ntt.Graph(stream)
        with g:
            for _ in range(100):
                step()
        gms, gkms = _time(lambda: g.replay(stream), stream, 20, 3)
        g.close()
        bfly = 3 * 4096 * 13
        _log("polymul8k: %.2f us/product per call (events %.2f us), %.2f us/product in a graph"
             % (ms * 1e3, kms * 1e3, gkms * 10))
        path = ("%d workgroups at once, then a recombination kernel" % (1 << split) if split
                else "one workgroup")
        return _line("single polymul mod p latency (Gbutterflies/s)", bfly / (ms * 1e-3) / 1e9, "Gbfly/s", ms, steps, 20,
                     {"workload": "one product mod 998244353 of two length-4096 operands, transform length 8192"},
                     {"us_per_product": round(ms * 1e3, 2), "events_us_per_call": round(kms * 1e3, 2),
                      "graph_us_per_product": round(gkms * 10, 2),
                      "path": path, "how": "polymul_modp calls on one stream; graph: 100 recorded calls per replay"})
    if name == "ntt2_24":
        p, x = inputs.ntt_2_24_inputs()
        plan = ntt.Plan(p, 24, 3, ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN)
        dx = ntt.to_device(x)
        n = 1 << 24

        def step():
            plan.forward(dx, out=dx, stream=stream)
            plan.inverse(dx, out=dx, stream=stream)
        steps = max(args.steps, 20)
        ms, kms = _time(step, stream, steps, 3)
        torch.cuda.synchronize()
        ok = bool(torch.equal(dx.cpu(), torch.from_numpy(x.view("int32"))))
        bfly = 2 * (n // 2) * 24
        alg = 4 * n * 4  # read + write of both transforms
        _log("ntt2_24: %.3f ms per forward+inverse (roundtrip identity %s)" % (ms, ok))
        return _line("forward+inverse NTT 2^24 (Gbutterflies/s)", bfly / (ms * 1e-3) / 1e9, "Gbfly/s", ms, steps, 3,
                     {"workload": "forward + inverse transform of length 2^24 mod 469762049, TFT order in between"},
                     {"roundtrip_identity": ok,
                      "hbm": {"algorithmic_bytes_per_step": alg, "achieved_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
                              "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                              "pass_bytes_per_step": 8 * n * 4},
                      "alu": _alu(bfly * SLOTS_PER_BFLY, ms)})
    if name == "intmul":
        a, b = inputs.intmul_inputs()
        da, db = ntt.to_device(a), ntt.to_device(b)
        dc = torch.empty(1 << 21, dtype=torch.int32, device="cuda")
        L = ntt.load()
        ws = torch.empty(L.intmul_workspace_bytes(a.size, b.size), dtype=torch.uint8, device="cuda")

        def step():
            ntt._check(L.intmul_crt(ntt._ptr(da), a.size, ntt._ptr(db), b.size, ntt._ptr(dc), ntt._ptr(ws), ws.numel(),
                                    ntt._stream(stream)), "intmul_crt")
        steps = max(args.steps, 10)
        ms, kms = _time(step, stream, steps, 2)
        N = 1 << 22
        bfly = 3 * 3 * (N // 2) * 22
        alg = 2 * (1 << 21) * 2 + (1 << 21) * 4
        _log("intmul: %.3f ms per product" % ms)
        return _line("three-prime integer product 2^25 x 2^25 bits (Gbutterflies/s)", bfly / (ms * 1e-3) / 1e9, "Gbfly/s",
                     ms, steps, 2,
                     {"workload": "product of two 2^21-limb (16-bit) integers, primes 998244353, 469762049, 167772161, transform length 2^22"},
                     {"ms_per_product": round(ms, 4),
                      "hbm": {"algorithmic_bytes_per_step": alg, "achieved_GBps": round(alg / (ms * 1e-3) / 1e9, 2)},
                      "alu": _alu(bfly * SLOTS_PER_BFLY, ms)})
    if name == "intmul32":
        # the same two integers as the integer-product configuration, in 32-bit chunks
        # (section 5.3's choice of h for these primes): transform length 2^21
        a, b = inputs.intmul_inputs()
        a32 = np.ascontiguousarray(a).view("<u4").astype(np.uint32)
        b32 = np.ascontiguousarray(b).view("<u4").astype(np.uint32)
        da, db = ntt.to_device(a32), ntt.to_device(b32)
        dc = torch.empty(a32.size + b32.size, dtype=torch.int32, device="cuda")
        L = ntt.load()
        ws = torch.empty(L.intmul32_workspace_bytes(a32.size, b32.size), dtype=torch.uint8, device="cuda")

        def step():
            ntt._check(L.intmul_crt32(ntt._ptr(da), a32.size, ntt._ptr(db), b32.size, ntt._ptr(dc), ntt._ptr(ws),
                                      ws.numel(), ntt._stream(stream)), "intmul_crt32")
        steps = max(args.steps, 10)
        ms, kms = _time(step, stream, steps, 2)
        N = 1 << 21
        bfly = 3 * 3 * (N // 2) * 21
        _log("intmul32: %.3f ms per product" % ms)
        return _line("three-prime integer product 2^25 x 2^25 bits, 32-bit chunks (Gbutterflies/s)",
                     bfly / (ms * 1e-3) / 1e9, "Gbfly/s", ms, steps, 2,
                     {"workload": "product of the same two 2^25-bit integers as 2^20 chunks of 32 bits (h = 32 by "
                                  "the chunk-size rule), primes 998244353, 469762049, 167772161, transform length 2^21"},
                     {"ms_per_product": round(ms, 4), "chunk_bits": ntt.intmul_chunk_bits(a.size, b.size),
                      "alu": _alu(bfly * SLOTS_PER_BFLY, ms),
                      "hbm": _hbm(2 * a32.size * 4 + (a32.size + b32.size) * 4, ms)})
    if name == "tft":
        # TFT truncation at sub-problem granularity: 1024 products mod 2013265921 of
        # operands of length 20000 (lc = 39999 <= 3 * 2^14: 3 of the 4 sub-problems of the
        # 2^16-point transform) beside the same batch at full length 2^15 (4 of 4)
        P = 2013265921
        res = {}
        for la in (20000, 1 << 15):
            _, A, B = inputs.polymul_batch_inputs(1024, la, P)
            dA, dB = ntt.to_device(A), ntt.to_device(B)
            dC = torch.empty((1024, 2 * la - 1), dtype=torch.int32, device="cuda")
            bt = ntt.Batch.rows(dA, dB, dC, P)
            ms, kms = _time(lambda: bt(stream), stream, max(args.steps, 50), 10)
            res[la] = kms
            del bt, dA, dB, dC
        full = 1024 * 3 * (1 << 15) * 16
        _log("tft: %.4f ms truncated, %.4f ms full" % (res[20000], res[1 << 15]))
        # Two-pass products truncated at row granularity (only ceil(lc / 2^L2) rows of the
        # row pass, the columns inverted by the inverse TFT; tuning key tft.rows = 1) against
        # the same products at full transform length (tft.rows = 0, the default)
        L = ntt.load()
        two = {}
        p62 = ntt.find_prime(62, 32)
        for (p, la) in ((998244353, 300000), (998244353, 600000), (2013265921, 140000), (p62, 300000)):
            a = ntt.to_device(inputs.residues(p, la, inputs.CFG_TEST, 31, 0))
            b = ntt.to_device(inputs.residues(p, la, inputs.CFG_TEST, 31, 1))
            c = torch.empty(2 * la - 1, dtype=a.dtype, device="cuda")
            ws = torch.empty(max(1, L.polymul_workspace_bytes(p, la, la)), dtype=torch.uint8, device="cuda")
            row = {}
            outs = {}
            for mode in (1, 0):
                ntt.tune_set("tft.rows.w%d" % ntt.word_bits(p), mode)
                ms2, kms2 = _time(lambda: ntt.polymul(a, b, p, out=c, stream=stream, workspace=ws), stream, 20, 3)
                row["truncated_ms" if mode else "full_length_ms"] = round(ms2, 4)
                outs[mode] = c.clone()
            ntt.tune_set("tft.rows.w%d" % ntt.word_bits(p), 0)  # the default: full length
            N = 1 << (2 * la - 2).bit_length()
            row.update({"p": p, "operand_len": la, "transform_len": N, "identical": bool(torch.equal(outs[0], outs[1])),
                        "time_ratio": round(row["truncated_ms"] / row["full_length_ms"], 4)})
            two["%d_%d" % (p, la)] = row
            _log("tft two-pass p=%d L=%d: %.4f ms truncated, %.4f ms full" % (p, la, row["truncated_ms"], row["full_length_ms"]))
        return _line("batched polymul with TFT truncation, 1024 x (20000 x 20000) mod 2013265921 (ms per launch)",
                     res[20000], "ms", res[20000], max(args.steps, 50), 10,
                     {"workload": "1024 products of length-20000 operands, transform length 2^16, 3 of 4 sub-problems"},
                     {"higher_is_better": False, "full_length_ms": round(res[1 << 15], 4),
                      "time_ratio": round(res[20000] / res[1 << 15], 4), "two_pass_single_products": two,
                      "note": "untruncated, both batches would take the same time (same transform length)"})
    if name == "polymatrix":
        return run_polymatrix(args)
    if name == "f64":
        return run_f64(args)
    if name == "fft":
        return run_fft(args)
    if name == "intmatrix":
        return run_intmatrix(args)
    if name == "serve":
        return run_serve(args)
    raise ValueError(name)


# Section 5.2's table of polynomial matrix products mod 469762049, degrees < 2^15
# (seconds on one core of the paper's machine), for context beside the times here
PAPER_POLYMATRIX_S = {1: 0.0012, 2: 0.0067, 4: 0.031, 8: 0.15, 16: 0.80, 32: 4.7}


def run_polymatrix(args):
    """n x n polynomial matrix products mod 469762049, degrees < 2^15 (transforms of
    2^16 words), n = 1 .. 32: transforms of the 2 n^2 entries, one n x n product per
    frequency, inverse transforms of the n^2 entries of C."""
    import torch

    from paper_1407_3383_amd import inputs, ntt
    stream = torch.cuda.Stream()
    p, d = 469762049, 1 << 15
    N, log2N = 1 << 16, 16
    L = ntt.load()
    rows = {}
    sizes = (1, 2, 4, 8, 16, 32) if not args.matrix_n else (args.matrix_n,)
    for n in sizes:
        A = inputs.residues(p, n * n * d, inputs.CFG_TEST, 77000 + n, 0)
        B = inputs.residues(p, n * n * d, inputs.CFG_TEST, 77000 + n, 1)
        dA = ntt.to_device(A).reshape(n, n, d)
        dB = ntt.to_device(B).reshape(n, n, d)
        dC = torch.empty((n, n, 2 * d - 1), dtype=torch.int32, device="cuda")
        ws = torch.empty(L.polymatmul_workspace_bytes(p, n, d), dtype=torch.uint8, device="cuda")

        def step():
            ntt._check(L.polymatmul_modp(p, n, ntt._ptr(dA), ntt._ptr(dB), d, ntt._ptr(dC), ntt._ptr(ws), ws.numel(),
                                         ntt._stream(stream)), "polymatmul_modp")
        steps = max(args.steps, 20)
        ms, kms = _time(step, stream, steps, 3)
        bfly = 3 * n * n * (N // 2) * log2N
        macs = n ** 3 * N
        alg = (2 * n * n * d + n * n * (2 * d - 1)) * 4
        rows[n] = {"ms": round(kms, 4), "Gbfly_per_s": round(bfly / (kms * 1e-3) / 1e9, 1),
                   "alu": _alu(bfly * SLOTS_PER_BFLY + macs, kms), "hbm": _hbm(alg, kms),
                   "Gmac_per_s": round(macs / (kms * 1e-3) / 1e9, 1),
                   "algorithmic_GBps": round(alg / (kms * 1e-3) / 1e9, 1),
                   "paper_cpu_s": PAPER_POLYMATRIX_S.get(n)}
        _log("polymatrix n=%d: %.4f ms (%.1f Gbfly/s)" % (n, kms, rows[n]["Gbfly_per_s"]))
        del dA, dB, dC, ws
    top = rows[max(rows)]
    return _line("polynomial matrix product %d x %d, degrees < 2^15, mod 469762049 (ms per product)" % (max(rows), max(rows)),
                 top["ms"], "ms", top["ms"], max(args.steps, 20), 3,
                 {"workload": "n x n polynomial matrices over F_p, p = 469762049, degrees < 2^15, transform length 2^16"},
                 {"higher_is_better": False, "by_n": rows,
                  "note": "paper_cpu_s: the section's table, one core of the paper's machine (context, not a target)"})


def run_serve(args):
    """Serving mix as the caller sees it: every product delivered to the request's host
    buffer.  Capacity with everything queued at t = 0, then Poisson arrivals at 0.5, 0.8
    and 0.95 of that capacity (p50/p99 latency from arrival to the product in host
    memory); the same with products left in device memory as a secondary figure."""
    import numpy as np
    import torch

    from paper_1407_3383_amd import inputs, ntt, serve
    p62 = ntt.find_prime(62, 32)
    primes = (998244353, 2013265921, p62)
    n = args.serve_requests
    specs = inputs.serve_requests(n, primes, 8.0, 20.0, 0)
    _log("serve: generating %d requests" % n)
    ops = [inputs.serve_operands(p, L, rid) for (p, L, rid) in specs]
    total_bfly = sum(serve.butterflies(L, L) for (_, L, _) in specs)
    bufs = {}  # result buffers by request id, allocated and touched once (the caller's buffers)

    def make(arrivals):
        reqs = [serve.Request(rid, p, a, b, arrival=float(t))
                for (p, L, rid), (a, b), t in zip(specs, ops, arrivals)]
        for r in reqs:
            r.result = bufs.get(r.rid)
        return reqs

    def keep(reqs):
        for r in reqs:
            if isinstance(r.result, np.ndarray):
                bufs[r.rid] = r.result

    budget = 8 << 30
    Server = serve.NativeServer

    def saturated(back, count):
        reqs = make([0.0] * count)
        srv = Server(budget, streams=4, max_batch=64, keep_results=back)
        wall = srv.run(reqs, realtime=False)
        srv.close()
        keep(reqs)
        return wall, srv

    def poisson(back, cap_rps, frac, reqs_fn=None):
        arr = inputs.poisson_arrivals(n, frac * cap_rps, int(frac * 100))
        reqs = (reqs_fn or make)(arr)
        srv = Server(budget, streams=4, max_batch=64, keep_results=back)
        w = srv.run(reqs, realtime=True)
        srv.close()
        keep(reqs)
        return w, srv

    # comparisons on the first m requests: the Python loop (which pins every queued
    # request's operands at once) and products copied straight into page-locked buffers
    m = min(n, 1000)
    warm = serve.Server(budget, streams=4, max_batch=64, keep_results=False)
    warm.run(make([0.0] * m), realtime=False)
    pysat = serve.Server(budget, streams=4, max_batch=64, keep_results=False)
    pywall = pysat.run(make([0.0] * m), realtime=False)
    _log("serve: python loop %.1f req/s over %d requests" % (m / pywall, m))
    # the native loop (ntt_server_*), products copied back: warm-up (allocates and touches
    # the result buffers), then the measured run
    saturated(True, n)
    wall, sat = saturated(True, n)
    capacity = n / wall
    _log("serve: native loop with copy-back %.1f req/s over %d requests" % (capacity, n))
    wall_dev, sat_dev = saturated(False, n)
    capacity_dev = n / wall_dev
    _log("serve: native loop, products left on the device %.1f req/s" % capacity_dev)
    pin = Server(budget, streams=4, max_batch=64, keep_results=True, pinned_results=True)
    wall_pin = pin.run(make([0.0] * m), realtime=False)
    pin.close()
    wall_sub, sub = saturated(True, m)
    out = {"metric": "serving mix with every product copied back to host memory: p50/p99 latency and throughput",
           "value": round(capacity, 2), "unit": "requests/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(wall * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32+u64", "data": "synthetic",
           "config": {"workload": "%d polymul requests, L = floor(2^U(8,20)), p uniform over {998244353, 2013265921, %d}, "
                                  "host operands in, host products out" % (n, p62),
                      "hbm_budget_bytes": budget, "streams": 4, "loop": "native (ntt_server_*)"},
           "saturated": {"requests_per_s": round(capacity, 2), "Gbfly_per_s": round(total_bfly / wall / 1e9, 2),
                         **serve.latency_stats(sat.completed)},
           "saturated_products_left_on_device": {"requests_per_s": round(capacity_dev, 2),
                                                 "Gbfly_per_s": round(total_bfly / wall_dev / 1e9, 2),
                                                 **serve.latency_stats(sat_dev.completed)},
           "first_%d_requests" % m: {
               "native_with_copy_back": {"requests_per_s": round(m / wall_sub, 2), **serve.latency_stats(sub.completed)},
               "native_with_copy_back_to_pinned": {"requests_per_s": round(m / wall_pin, 2),
                                                   **serve.latency_stats(pin.completed)},
               "python_loop_products_left_on_device": {"requests_per_s": round(m / pywall, 2),
                                                       **serve.latency_stats(pysat.completed)}}}
    levels, levels_dev = {}, {}
    for frac in (0.5, 0.8, 0.95):
        for back, cap_rps, dst in ((True, capacity, levels), (False, capacity_dev, levels_dev)):
            w, srv = poisson(back, cap_rps, frac)
            st = serve.latency_stats(srv.completed)
            dst[str(frac)] = {"offered_rps": round(frac * cap_rps, 2), "achieved_rps": round(n / w, 2),
                              "Gbfly_per_s": round(total_bfly / w / 1e9, 2),
                              "max_inflight_batches": srv.max_inflight_batches, **st}
            _log("serve at %.2f x capacity (%s): p50 %.3f ms, p99 %.3f ms"
                 % (frac, "copy-back" if back else "device", st["p50_ms"], st["p99_ms"]))
    out["poisson"] = levels
    out["poisson_products_left_on_device"] = levels_dev

    # the same stream with every 10th request an integer product of L 16-bit limbs
    # (three-prime transform, CRT and carries), at 0.8 of the capacity, copied back
    def make_mixed(arrivals):
        reqs = make(arrivals)
        for k in range(0, n, 10):
            r = reqs[k]
            L = r.a.size
            a = inputs.limbs16(L, inputs.CFG_SERVE, r.rid, 0)
            b = inputs.limbs16(L, inputs.CFG_SERVE, r.rid, 1)
            reqs[k] = serve.Request(r.rid, 0, a, b, arrival=r.arrival, kind="int")
        return reqs
    warm = Server(budget, streams=4, max_batch=64, keep_results=True)
    warm.run(make_mixed([0.0] * n), realtime=False)
    warm.close()
    w, srv = poisson(True, capacity, 0.8, make_mixed)
    st = serve.latency_stats(srv.completed)
    ints = [r for r in srv.completed if r.kind == "int"]
    out["with_integer_products"] = {"share": 0.1, "offered_rps": round(0.8 * capacity, 2), "achieved_rps": round(n / w, 2),
                                    "integer_requests": len(ints), "integer_p50_p99_ms": [
                                        serve.latency_stats(ints)["p50_ms"], serve.latency_stats(ints)["p99_ms"]], **st}
    _log("serve with integer products: p50 %.3f ms, p99 %.3f ms" % (st["p50_ms"], st["p99_ms"]))
    torch.cuda.synchronize()
    return out


def run_f64(args):
    """Section 3's numeric-type arithmetic against the 64-bit integer words: 1024
    products of length-2^14 operands (transform length 2^15, the fused kernel's 64-bit
    limit) modulo the largest primes below 2^48, 2^49 and 2^50 with 2^20 | p - 1, 8192
    products of length 2^11, and 16 products of length-2^19 operands (two-pass
    transforms of length 2^20), once with residues in doubles (Function 16) and once in
    64-bit integers (Function 8 over 64-bit words), same kernels otherwise."""
    import torch

    from paper_1407_3383_amd import inputs, ntt
    stream = torch.cuda.Stream()
    res = {}
    for bits, items, n in ((48, 1024, 1 << 14), (49, 1024, 1 << 14), (50, 1024, 1 << 14), (49, 8192, 1 << 11),
                           (49, 16, 1 << 19), (50, 16, 1 << 19)):
        N = 2 * n
        log2N = N.bit_length() - 1
        bfly = items * 3 * (N // 2) * log2N
        p = ntt.find_prime(bits, 20)
        _, A, B = inputs.polymul_batch_inputs(items, n, p)
        dA, dB = ntt.to_device(A), ntt.to_device(B)
        C = torch.empty((items, 2 * n - 1), dtype=torch.int64, device="cuda")
        bt = ntt.Batch.rows(dA, dB, C, p)
        _, ims = _time(lambda: bt(stream), stream, max(args.steps, 20), 3)
        Af, Bf = dA.double(), dB.double()
        Cf = torch.empty((items, 2 * n - 1), dtype=torch.float64, device="cuda")
        bf = ntt.Batch.rows(Af, Bf, Cf, p, f64=True)
        _, fms = _time(lambda: bf(stream), stream, max(args.steps, 20), 3)
        torch.cuda.synchronize()
        same = bool(torch.equal(Cf.to(torch.int64), C))
        res["%d-bit p, %d x 2^%d" % (bits, items, log2N - 1)] = {"p": p, "u64_ms": round(ims, 4), "f64_ms": round(fms, 4),
                     "u64_Gbfly_per_s": round(bfly / (ims * 1e-3) / 1e9, 1),
                     "f64_Gbfly_per_s": round(bfly / (fms * 1e-3) / 1e9, 1),
                     "f64_over_u64_speed": round(ims / fms, 3), "identical_results": same}
        _log("f64 %d-bit prime, %d x 2^%d: u64 %.4f ms, f64 %.4f ms, identical %s"
             % (bits, items, log2N - 1, ims, fms, same))
        bt.close()
        bf.close()
        del dA, dB, C, Af, Bf, Cf, bt, bf
    top = res["49-bit p, 1024 x 2^14"]
    return _line("batched polymul with FP64 residues, 1024 x (2^14 x 2^14) mod a 49-bit prime (Gbutterflies/s)",
                 top["f64_Gbfly_per_s"], "Gbfly/s", top["f64_ms"], max(args.steps, 20), 3,
                 {"workload": "1024 products of length-2^14 operands, transform length 2^15, p < 2^49 and p < 2^48"},
                 {"dtype": "f64", "by_case": res,
                  "note": "u64: the same batch with 64-bit integer residues (Function 8 over 64-bit words)"})


# Section 5.1's tables of transform times of one core of the paper's machine (microseconds,
# its AVX rows): length 2^8..2^20 over Z/469762049Z (32-bit words, Barrett) and over
# Z/1108307720798209Z (doubles, FMA), for context beside the times here
PAPER_FFT32_US = {8: 0.64, 9: 1.4, 10: 2.9, 11: 6.4, 12: 14, 13: 30, 14: 64, 15: 140, 16: 290, 17: 630, 18: 1400,
                  19: 3000, 20: 6800}
PAPER_FFT64_US = {8: 1.2, 9: 2.5, 10: 5.6, 11: 12, 12: 26, 13: 57, 14: 120, 15: 270, 16: 580, 17: 1200, 18: 2600,
                  19: 6100, 20: 15000}


def run_fft(args):
    """Forward transforms of length 2^8..2^20 (section 5.1's two tables): mod 469762049
    in 32-bit words, and mod 1108307720798209 = 63 * 2^44 + 1 once in 64-bit integer
    words and once in doubles (NTT_FP64).  Per length: one transform alone (latency) and a
    batch of 2^24 / n transforms in one call (throughput); TFT order out, as the paper's
    FFTs leave it."""
    import numpy as np
    import torch

    from paper_1407_3383_amd import inputs, ntt
    stream = torch.cuda.Stream()
    p32, p64 = 469762049, 63 * 2 ** 44 + 1
    total = 1 << 24
    res = {}
    flags = ntt.NTT_BITREV_OUT
    steps = max(args.steps, 20)
    for log2n in range(8, 21):
        n = 1 << log2n
        batch = total // n
        row = {"paper_us_32": PAPER_FFT32_US[log2n], "paper_us_fp64": PAPER_FFT64_US[log2n]}
        ref64 = None
        for kind, p, fl in (("u32", p32, flags), ("u64", p64, flags), ("f64", p64, flags | ntt.NTT_FP64)):
            plan = ntt.Plan(p, log2n, 0, fl)
            x = inputs.residues(p, total, inputs.CFG_FFT, log2n)
            dx = torch.from_numpy(x.astype(np.float64)).cuda() if kind == "f64" else ntt.to_device(x)
            dy = torch.empty_like(dx)
            ws = ntt._workspace(max(plan.workspace_bytes(batch), 1), dx.device)
            _, one_ms = _time(lambda: plan.forward(dx, out=dy, batch=1, stream=stream, workspace=ws), stream, steps, 3)
            _, all_ms = _time(lambda: plan.forward(dx, out=dy, batch=batch, stream=stream, workspace=ws), stream,
                              max(steps // 4, 5), 2)
            torch.cuda.synchronize()
            bfly = batch * (n // 2) * log2n
            row[kind] = {"one_us": round(one_ms * 1e3, 2), "batch": batch, "batch_ms": round(all_ms, 4),
                         "us_per_transform_in_batch": round(all_ms * 1e3 / batch, 4),
                         "Gbfly_per_s": round(bfly / (all_ms * 1e-3) / 1e9, 1)}
            if kind == "u64":
                ref64 = dy.cpu().numpy()
            elif kind == "f64":
                row["f64_equals_u64"] = bool((dy.cpu().numpy().astype(np.uint64) == ref64.astype(np.uint64)).all())
            plan.close()
            del dx, dy, ws
        res["2^%d" % log2n] = row
        _log("fft 2^%d: u32 %.2f us / %.4f us per transform in a batch; u64 %.2f / %.4f; f64 %.2f / %.4f; f64 = u64 %s"
             % (log2n, row["u32"]["one_us"], row["u32"]["us_per_transform_in_batch"], row["u64"]["one_us"],
                row["u64"]["us_per_transform_in_batch"], row["f64"]["one_us"], row["f64"]["us_per_transform_in_batch"],
                row["f64_equals_u64"]))
    top = res["2^20"]
    return _line("forward FFT over Z/1108307720798209Z, length 2^20, residues in doubles (Gbutterflies/s)",
                 top["f64"]["Gbfly_per_s"], "Gbfly/s", top["f64"]["batch_ms"], max(steps // 4, 5), 2,
                 {"workload": "forward transforms of length 2^8..2^20, 2^24 / n per call, mod 469762049 (32-bit words) "
                              "and mod 1108307720798209 (64-bit words and doubles)"},
                 {"dtype": "f64", "by_length": res,
                  "note": "one_us: a single transform per call; batch: 2^24 / n transforms per call; paper_us: one "
                          "core of the paper's machine (AVX rows), context only"})


# Section 5.3's table of integer matrix products in bit-size 32 x 2^15 (seconds on one
# core of the paper's machine), for context beside the times here
PAPER_INTMATRIX_S = {1: 0.0060, 2: 0.022, 4: 0.095, 8: 0.44, 16: 2.3, 32: 13}


def run_intmatrix(args):
    """n x n integer matrix products, entries of 32 x 2^15 bits (2^15 chunks of 32
    bits): three polynomial matrix products of transform length 2^16 and a batched CRT
    tail, n = 1 .. 32."""
    import torch

    from paper_1407_3383_amd import inputs, ntt
    stream = torch.cuda.Stream()
    na = 1 << 15
    L = ntt.load()
    rows = {}
    sizes = (1, 2, 4, 8, 16, 32) if not args.matrix_n else (args.matrix_n,)
    for n in sizes:
        A = inputs.limbs32(n * n * na, inputs.CFG_TEST, 88000 + n, 0)
        B = inputs.limbs32(n * n * na, inputs.CFG_TEST, 88000 + n, 1)
        dA = ntt.to_device(A).reshape(n, n, na)
        dB = ntt.to_device(B).reshape(n, n, na)
        dC = torch.empty((n, n, 2 * na + 1), dtype=torch.int32, device="cuda")
        ws = torch.empty(L.intmatmul32_workspace_bytes(n, na), dtype=torch.uint8, device="cuda")

        def step():
            ntt._check(L.intmatmul_crt32(n, ntt._ptr(dA), ntt._ptr(dB), na, ntt._ptr(dC), ntt._ptr(ws), ws.numel(),
                                         ntt._stream(stream)), "intmatmul_crt32")
        _, kms = _time(step, stream, max(args.steps, 10), 2)
        N = 1 << 16
        bfly = 3 * 3 * n * n * (N // 2) * 16
        macs = 3 * n ** 3 * N
        alg = (2 * n * n * na + n * n * (2 * na + 1)) * 4
        rows[n] = {"ms": round(kms, 4), "alu": _alu(bfly * SLOTS_PER_BFLY + macs, kms), "hbm": _hbm(alg, kms),
                   "paper_cpu_s": PAPER_INTMATRIX_S.get(n)}
        _log("intmatrix n=%d: %.4f ms" % (n, kms))
        del dA, dB, dC, ws
    top = rows[max(rows)]
    return _line("integer matrix product %d x %d, entries of 32 x 2^15 bits (ms per product)" % (max(rows), max(rows)),
                 top["ms"], "ms", top["ms"], max(args.steps, 10), 2,
                 {"workload": "n x n matrices of 2^20-bit integers, 32-bit chunks, primes 998244353, 469762049, "
                              "167772161, transform length 2^16"},
                 {"higher_is_better": False, "by_n": rows,
                  "note": "paper_cpu_s: the section's table, one core of the paper's machine (context, not a target)"})
