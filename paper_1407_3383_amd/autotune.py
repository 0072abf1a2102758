"""Autotuner for the launch-shape choices of the HIP library on one GPU.

The choices (keys of ``ntt_tune_set``, see include/ntt_mi355x.h):

* ``split.w<W>.L<L>``: row length 2^L2 of a two-pass transform of length 2^L
  (Algorithm 1 read as 2^(L-L2) rows of 2^L2 words): 12, 13 or 14
  for 32-bit primes, 12 or 13 for 64-bit ones.  Shorter rows give more workgroups
  per CU in the row pass but longer columns in the column pass.
* ``psplit.w<W>.L<L>``: the same for the plans of the products (the row pass there is
  the fused twist / forward x2 / entry-wise product / inverse kernel).
* ``fused.single.max.w<W>``: up to which transform length a single product runs in
  the one-workgroup fused kernel rather than the two-pass path (many workgroups).
* ``single.split.w<W>.L<L>``: whether a single product of length 2^L runs its 2^d
  sub-problems on 2^d workgroups at once (the latency path), and with which d.

Every candidate is timed with HIP events on its own stream, and every candidate's
output is compared with the first candidate's (they must be identical: the results
are canonical residues).  The choices are written as ``key value`` lines, with the
timings in comments, to the file the binding loads with the library.

    python -m paper_1407_3383_amd.autotune [--out FILE] [--reps R] [--quick]
"""
from __future__ import annotations

import argparse
import datetime
import os
import sys
import time

import numpy as np

from . import inputs, ntt

PRIMES = {32: 469762049, 64: 4611685941117976577}       # transforms (2-adic orders 26 and 33)
PRODUCT_PRIMES = {32: 998244353, 64: 4611685941117976577}
SPLITS = {32: (14, 13, 12), 64: (13, 12)}
TRANSFORM_L = {32: range(15, 25), 64: range(14, 22)}
PRODUCT_L = {32: range(15, 24), 64: range(14, 22)}
FUSED_L = {32: (15, 16), 64: (14, 15)}
SPLIT_L = {32: range(11, 17), 64: range(11, 16)}
SEED_ITEM = 4242


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _time(fn, stream, reps: int) -> float:
    """Mean milliseconds of fn() over `reps` calls, after warm-up calls (at least 50 ms
    of them, so that the GPU clocks have ramped up)."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.05:
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _same(results, what):
    ref = results[0]
    for r in results[1:]:
        if not np.array_equal(r, ref):
            raise RuntimeError("candidates disagree on %s" % what)


def tune_transform(wb: int, L: int, reps: int, stream):
    """Best row length of a forward + inverse pair of length 2^L."""
    import torch
    p = PRIMES[wb]
    x = ntt.to_device(inputs.residues(p, 1 << L, inputs.CFG_TEST, SEED_ITEM + L))
    y, z = torch.empty_like(x), torch.empty_like(x)
    times, outs = {}, []
    key = "split.w%d.L%d" % (wb, L)
    for cand in SPLITS[wb]:
        ntt.tune_set(key, cand)
        plan = ntt.Plan(p, L, flags=ntt.NTT_BITREV_OUT | ntt.NTT_BITREV_IN)
        assert plan.info.row_log2 == cand, (plan.info.row_log2, cand)
        ws = torch.empty(max(ntt.load().ntt_workspace_bytes(plan.handle, 1), 1), dtype=torch.uint8, device="cuda")

        def step():
            plan.forward(x, out=y, stream=stream, workspace=ws)
            plan.inverse(y, out=z, stream=stream, workspace=ws)
        times[cand] = _time(step, stream, reps)
        torch.cuda.synchronize()
        if not torch.equal(z, x):
            raise RuntimeError("%s = %d: inverse(forward(x)) != x" % (key, cand))
        outs.append(ntt.to_numpy(y))
        plan.close()
    _same(outs, key)
    return key, min(times, key=times.get), times


def tune_product(wb: int, L: int, reps: int, stream):
    """Best row length of the two-pass product with transform length 2^L."""
    import torch
    p = PRODUCT_PRIMES[wb]
    n = 1 << (L - 1)
    a = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + L, 0))
    b = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + L, 1))
    c = torch.empty(2 * n - 1, dtype=a.dtype, device="cuda")
    ws = torch.empty(max(ntt.load().polymul_workspace_bytes(p, n, n), 1), dtype=torch.uint8, device="cuda")
    times, outs = {}, []
    key = "psplit.w%d.L%d" % (wb, L)
    for cand in SPLITS[wb]:
        ntt.tune_set(key, cand)
        ntt.plan_cache_clear()
        times[cand] = _time(lambda: ntt.polymul(a, b, p, out=c, stream=stream, workspace=ws), stream, reps)
        outs.append(ntt.to_numpy(c))
    _same(outs, key)
    return key, min(times, key=times.get), times


def tune_single_fused(wb: int, reps: int, stream):
    """Largest log2 N at which one product is faster in the fused kernel."""
    import torch
    p = PRODUCT_PRIMES[wb]
    key = "fused.single.max.w%d" % wb
    lo = FUSED_L[wb][0] - 1
    best = lo
    times = {}
    for L in FUSED_L[wb]:
        n = 1 << (L - 1)
        a = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + 100 + L, 0))
        b = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + 100 + L, 1))
        c = torch.empty(2 * n - 1, dtype=a.dtype, device="cuda")
        res = {}
        outs = []
        for mode, val in (("fused", FUSED_L[wb][-1]), ("two-pass", lo)):
            ntt.tune_set(key, val)
            ws = torch.empty(max(ntt.load().polymul_workspace_bytes(p, n, n), 1), dtype=torch.uint8, device="cuda")
            res[mode] = _time(lambda: ntt.polymul(a, b, p, out=c, stream=stream, workspace=ws), stream, reps)
            outs.append(ntt.to_numpy(c))
        _same(outs, "%s at 2^%d" % (key, L))
        times[L] = res
        if res["fused"] <= res["two-pass"] and best == L - 1:
            best = L
    return key, best, times


def tune_single_split(wb: int, L: int, reps: int, stream):
    """Depth d of the split latency path for one product of length 2^L (0: not split)."""
    import torch
    p = PRODUCT_PRIMES[wb]
    n = 1 << (L - 1)
    a = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + 200 + L, 0))
    b = ntt.to_device(inputs.residues(p, n, inputs.CFG_TEST, SEED_ITEM + 200 + L, 1))
    c = torch.empty(2 * n - 1, dtype=a.dtype, device="cuda")
    key = "single.split.w%d.L%d" % (wb, L)
    times, outs = {}, []
    for d in (0, 1, 2, 3):
        if d and not 10 <= L - d <= (13 if wb == 32 else 12):
            continue
        ntt.tune_set(key, d)
        ws = torch.empty(max(ntt.load().polymul_workspace_bytes(p, n, n), 1), dtype=torch.uint8, device="cuda")
        times[d] = _time(lambda: ntt.polymul(a, b, p, out=c, stream=stream, workspace=ws), stream, reps)
        outs.append(ntt.to_numpy(c))
    _same(outs, key)
    return key, min(times, key=times.get), times


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=ntt.TUNE_FILE)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--quick", action="store_true", help="a few sizes only (a check of the tuner itself)")
    args = ap.parse_args(argv)
    os.environ["NTT_TUNE_FILE"] = ""  # start from the built-in defaults
    import torch
    ntt.load()
    ntt.tune_clear()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    props = torch.cuda.get_device_properties(0)
    lines = ["# launch-shape choices for %s (%s, %d CUs), written by paper_1407_3383_amd.autotune on %s"
             % (props.name, getattr(props, "gcnArchName", "?"), props.multi_processor_count,
                datetime.date.today().isoformat()),
             "# key value   # mean ms per candidate"]
    t0 = time.time()
    jobs = []
    for wb in (32, 64):
        Ls = list(TRANSFORM_L[wb])
        Ps = list(PRODUCT_L[wb])
        Ss = list(SPLIT_L[wb])
        if args.quick:
            Ls, Ps, Ss = Ls[:1] + Ls[-1:], Ps[:1], Ss[2:3]
        # the single-product threshold and split depths first: they decide which
        # product sizes take the two-pass path whose row length is tuned next
        jobs += ([("t", wb, L) for L in Ls] + [("f", wb, 0)] + [("s", wb, L) for L in Ss]
                 + [("p", wb, L) for L in Ps])
    with torch.cuda.stream(stream):
        for kind, wb, L in jobs:
            if kind == "t":
                key, best, times = tune_transform(wb, L, args.reps, stream)
            elif kind == "p":
                key, best, times = tune_product(wb, L, args.reps, stream)
            elif kind == "s":
                key, best, times = tune_single_split(wb, L, args.reps, stream)
            else:
                key, best, times = tune_single_fused(wb, args.reps, stream)
            ntt.tune_set(key, best)
            ntt.plan_cache_clear()
            desc = ", ".join("%s: %s" % (k, ("%.4f" % v) if isinstance(v, float) else
                                          "/".join("%s %.4f" % kv for kv in v.items()))
                             for k, v in times.items())
            lines.append("%-24s %d   # %s" % (key, best, desc))
            _log("%s -> %d (%s)  [%.0f s]" % (key, best, desc, time.time() - t0))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    _log("wrote %s" % args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
