#!/usr/bin/env python3
"""Benchmark of the batched polynomial product mod p on one MI355X.

Workload: 1024 independent products mod p = 2013265921 (15 * 2^27 + 1), both operands
of length 2^15 with uniform residues, transform length 2^16 (section 5.2's product:
two forward transforms, entry-wise product, one inverse), all in one fused launch.
A step is one such batched launch with the operands already resident in HBM.

Printed (one JSON line): radix-2-equivalent butterflies per second over the three
transforms of every product, the HBM traffic rate on algorithmic bytes, the roofline
of the fused kernel (it is bound by the integer VALU), the same products issued as
1024 separate per-call launches, and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]   (defaults: 100 timed steps, 30 warm-up)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NTT polymul mod p: Gbutterflies/s, % HBM roofline, batched vs per-call"
P = 2013265921
HBM_PEAK_GBPS = 8000.0
# Integer-VALU ceiling of the butterflies, from the chip's unit counts and clock:
# 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue one lane-operation per lane and clock
# for 32-bit multiplies, multiply-adds and min (39.3 T/s) and two for plain 32-bit
# add and subtract (78.6 T/s), as measured by paper_1407_3383_amd.valu_rates.  The
# butterfly of this workload's 31-bit prime (every sum formed from reduced operands,
# since 2p < 2^32 < 4p) issues a high product, two multiply-adds and two mins (5 full-
# rate slots) plus five adds and subtracts (2.5 slots): at most 256 * 64 * 2.4e9 / 7.5
# = 5.24 T butterflies/s.  The same butterflies on registers alone measure 4.1 T/s.
ALU_SLOTS_PER_BFLY = 7.5
BFLY_PEAK_G = 256 * 64 * 2.4e9 / ALU_SLOTS_PER_BFLY / 1e9
BFLY_REGISTERS_G = 4129.0  # CT butterfly of this prime on registers alone (profiles/valu_rates.md)
# HBM bytes per launch of the fused kernel at the default workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE counter runs scaled by a plain copy's readings; valid only
# while the kernel's sources are the ones that were measured.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "polymul_fused_kernel_batch1024_n65536.md")
KERNEL_SOURCES = ["arith.hpp", "common.hpp", "kernels.hpp", "ntt_lds.hpp", "ntt_wave.hpp", "polymul_fused.hpp", "kernels_poly_w32c3.hip"]


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def settle(step, seconds: float):
    """Untimed launches of `step` for about `seconds` of wall time."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            step()
        torch.cuda.synchronize()


def measured_traffic():
    """(bytes per launch, None) from the committed counter summary, or (None, reason)."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None, "no counter summary"
    t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    hsh = re.search(r"^kernel_sources_sha256: ([0-9a-f]+)", text, re.M)
    if not t or not hsh:
        return None, "counter summary without figures"
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1407_3383_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != hsh.group(1):
        return None, "kernel changed since the counters were taken"
    return int(t.group(1)), None


def host_cores() -> int:
    """Host threads for the all-cores oracle leg (at most 16: one GPU's share of a box)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_leg(A, B, C, items: int, threads: int, seconds: float, first: int):
    """The oracle's product of items first, first + 1, ... (in a scrambled order,
    wrapping around the batch) on `threads` threads for about `seconds`, each compared
    with the GPU's product."""
    import concurrent.futures as cf
    import threading

    import numpy as np

    import oracle
    order = [((first + k) * 97) % items for k in range(64 * items)]
    lock = threading.Lock()
    state = {"next": 0, "done": 0, "mismatches": 0}
    t0 = time.perf_counter()

    def worker():
        while time.perf_counter() - t0 < seconds:
            with lock:
                if state["next"] >= len(order):
                    return
                i = order[state["next"]]
                state["next"] += 1
            ref = oracle.polymul_ntt(A[i], B[i], P, 31)
            bad = int(not np.array_equal(ref, C[i].astype(np.uint64)))
            with lock:
                state["done"] += 1
                state["mismatches"] += bad

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for f in [ex.submit(worker) for _ in range(threads)]:
            f.result()
    return {"done": state["done"], "mismatches": state["mismatches"], "seconds": time.perf_counter() - t0,
            "threads": threads}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--settle-seconds", type=float, default=0.5,
                    help="untimed launches before the warm-up steps while the GPU clocks ramp up")
    ap.add_argument("--items", type=int, default=1024)
    ap.add_argument("--log2len", type=int, default=15)
    ap.add_argument("--percall-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-percall", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "polymul8k", "ntt2_24", "intmul", "intmul32", "tft", "polymatrix", "intmatrix", "f64", "fft", "serve", "all"],
                    help="batch (default, the headline line) or one of the other configurations")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--matrix-n", type=int, default=0, help="polymatrix, intmatrix: one matrix size only (default 1 .. 32)")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="a tuning choice of the library (ntt_tune_set) applied before the run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the products shard trivially across GPUs; see the design notes).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1407_3383_amd import inputs, ntt

    torch.cuda.set_device(0)
    for kv in args.tune:
        key, val = kv.split("=", 1)
        ntt.tune_set(key, int(val))
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 18  # int32 words
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB three times" % args.copy_calibration_mib)
        return 0
    if args.workload != "batch":
        import bench_workloads
        names = (["polymul8k", "ntt2_24", "intmul", "intmul32", "tft", "polymatrix", "intmatrix", "f64", "fft", "serve"] if args.workload == "all"
                 else [args.workload])
        for name in names:
            print(json.dumps(bench_workloads.run(name, args)), flush=True)
        return 0
    items, L = args.items, 1 << args.log2len
    L_len = L
    lc = 2 * L - 1
    log2N = (lc - 1).bit_length()
    N = 1 << log2N
    bfly_per_item = 3 * (N // 2) * log2N
    bfly_per_step = items * bfly_per_item
    alg_bytes = items * (2 * L * 4 + lc * 4)

    log("generating %d x 2 operands of length %d" % (items, L))
    _, A, B = inputs.polymul_batch_inputs(items, L, P)
    dA, dB = ntt.to_device(A), ntt.to_device(B)
    dC = torch.empty((items, lc), dtype=torch.int32, device="cuda")
    batch = ntt.Batch.rows(dA, dB, dC, P)
    stream = torch.cuda.Stream()

    # The first tens of launches on an idle GPU run ~10% slower while its clocks ramp
    # up: settle them with untimed launches before the warm-up steps.
    log("settling clocks for %.1f s, then warmup %d" % (args.settle_seconds, args.warmup))
    settle(lambda: batch(stream), args.settle_seconds)
    for _ in range(args.warmup):
        batch(stream)
    torch.cuda.synchronize()

    log("timing %d steps" % args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        batch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = e0.elapsed_time(e1) / args.steps  # one fused kernel per step
    ms_per_step = wall * 1e3 / args.steps
    value = bfly_per_step / (ms_per_step * 1e-3) / 1e9
    log("batched: %.3f ms/step (events %.3f ms/kernel), %.1f Gbfly/s" % (ms_per_step, kern_ms, value))
    # the batched launch's products, read back before anything else writes to the device
    C = ntt.to_numpy(dC)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gbfly/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "batched polymul: %d products mod %d, operands of length %d, transform length %d, one fused launch"
                        % (items, P, L, N),
            "items": items, "operand_len": L, "ntt_len": N, "p": P,
            **({"tuning": dict(kv.split("=", 1) for kv in args.tune)} if args.tune else {}),
        },
        "hbm": {
            "algorithmic_bytes_per_step": alg_bytes,
            "achieved_GBps": round(alg_bytes / (ms_per_step * 1e-3) / 1e9, 2),
            "peak_GBps": HBM_PEAK_GBPS,
            "frac": round(alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        },
    }
    achieved_g = bfly_per_step / (kern_ms * 1e-3) / 1e9
    traffic, why = (measured_traffic() if (items, args.log2len) == (1024, 15) and not args.tune
                    else (None, "not the profiled workload"))
    out["roofline"] = {
        "bound": "alu",
        "kernel": "polymul_fused_kernel<u32, 1024 threads, 2^14-word sub-problems>",
        "achieved": round(achieved_g, 1),
        "peak": round(BFLY_PEAK_G, 1),
        "unit": "Gbfly/s (kernel time; peak = 256 CUs x 64 lanes x 2.4 GHz / %.1f issue slots per butterfly of "
                "this prime)" % ALU_SLOTS_PER_BFLY,
        "frac": round(achieved_g / BFLY_PEAK_G, 4),
        "traffic": traffic,
        "kernel_ms": round(kern_ms, 4),
        "registers_only_bfly": BFLY_REGISTERS_G,
        "frac_of_registers_only": round(achieved_g / BFLY_REGISTERS_G, 4),
    }
    if traffic is None:
        out["roofline"]["traffic_note"] = why
    else:
        out["roofline"]["traffic_note"] = ("HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, "
                                           "%.2fx the algorithmic bytes)" % (traffic / alg_bytes))

    if not args.no_percall:
        # The same products as separate polymul_modp calls (each on its own launch
        # shape: the tuned single-product path), with the workspace allocated once.
        # Host-issued calls include the per-call host cost; the device time comes
        # from the same calls recorded in one HIP graph and replayed.
        log("per-call baseline: %d separate polymul_modp calls" % items)
        lib = ntt.load()
        ws1 = torch.empty(max(lib.polymul_workspace_bytes(P, L_len, L_len), 1), dtype=torch.uint8, device="cuda")
        dC1 = torch.full_like(dC, -1)  # the per-call products go to their own buffer
        rows = [(dA[i], dB[i], dC1[i]) for i in range(items)]

        def one(a, b, c):
            ntt._check(lib.polymul_modp(P, ntt._ptr(a), L_len, ntt._ptr(b), L_len, ntt._ptr(c), ntt._ptr(ws1),
                                      ws1.numel(), ntt._stream(stream)), "polymul_modp")
        settle(lambda: one(*rows[0]), 0.2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.percall_steps):
            for a, b, c in rows:
                one(a, b, c)
        torch.cuda.synchronize()
        pc_ms = (time.perf_counter() - t0) * 1e3 / args.percall_steps
        g = ntt.Graph(stream)
        with g:
            for a, b, c in rows:
                one(a, b, c)
        g.replay(stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            g.replay(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        pcg_ms = e0.elapsed_time(e1) / 3
        g.close()
        same = bool(np.array_equal(ntt.to_numpy(dC1), C))
        del dC1
        out["per_call"] = {
            "ms_per_step": round(pc_ms, 3),
            "value": round(bfly_per_step / (pc_ms * 1e-3) / 1e9, 3),
            "unit": "Gbfly/s",
            "batched_speedup": round(pc_ms / ms_per_step, 2),
            "graph_ms_per_step": round(pcg_ms, 3),
            "graph_value": round(bfly_per_step / (pcg_ms * 1e-3) / 1e9, 3),
            "batched_speedup_vs_graph": round(pcg_ms / ms_per_step, 2),
            "how": ("the same %d products as %d polymul_modp calls on one stream (workspace allocated once); "
                    "graph: the %d calls recorded in one HIP graph, device time" % (items, items, items)),
            "identical_to_batched": same,
        }
        if not same:
            log("WARNING: per-call products differ from the batched launch's")
        log("per-call: %.2f ms/step host-issued, %.2f ms/step as one graph" % (pc_ms, pcg_ms))

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle transform product on sampled items, ~%.0f s on one core, then ~%.0f s on %d cores"
            % (args.cpu_seconds, args.cpu_seconds, host_cores()))
        one = oracle_leg(A, B, C, items, 1, args.cpu_seconds, 0)
        many = oracle_leg(A, B, C, items, host_cores(), args.cpu_seconds, one["done"])
        out["cpu_baseline"] = {
            "value": round(one["done"] * bfly_per_item / one["seconds"] / 1e9, 6),
            "unit": "Gbfly/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "%d of the %d products of the batched launch (textbook radix-2 transforms, __int128 %% "
                      "reductions), %.1f s on one host core" % (one["done"], items, one["seconds"]),
            "gpu_vs_oracle_mismatches": one["mismatches"],
            "all_cores": {
                "value": round(many["done"] * bfly_per_item / many["seconds"] / 1e9, 6),
                "cores": many["threads"],
                "sample": "%d products of the batch (continuing the sample, wrapping around), independent "
                          "products on %d threads (the oracle's C routine releases the GIL), %.1f s"
                          % (many["done"], many["threads"], many["seconds"]),
                "gpu_vs_oracle_mismatches": many["mismatches"],
            },
        }
        if one["mismatches"] or many["mismatches"]:
            log("WARNING: %d sampled products differ from the oracle" % (one["mismatches"] + many["mismatches"]))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
