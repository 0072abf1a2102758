"""Issue rates of the vector ALU instructions the transform kernels are made of, and
of the kernels' own butterflies on registers alone, measured on the current GPU.

Each probe (``csrc/valu_rates.hip``) runs 8 independent chains of one instruction
per thread (inline assembly, so nothing is merged or dropped) over many waves per
SIMD; the rate is the instructions issued divided by the kernel's duration (HIP
events on the launch stream).  The butterfly probes run the library's CT and GS
butterflies (31-bit prime: every sum formed from reduced operands; p < 2^30: the
lazy ranges) with a twiddle held in scalar registers, which is the butterfly of the
wave-uniform rounds, and report butterflies per second.  These are the ceilings the
product kernels are measured against.

    python -m paper_1407_3383_amd.valu_rates [--iters N] [--grid G] [--json FILE]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvalu_rates.so")

# (name, op code, kind, lane-ops or butterflies per iteration per thread)
PROBES = [
    ("v_add_u32", 0, "op"), ("v_sub_u32", 1, "op"), ("v_add3_u32", 2, "op"), ("v_min_u32", 3, "op"),
    ("v_mul_lo_u32", 4, "op"), ("v_mul_hi_u32", 5, "op"), ("v_mad_u64_u32", 6, "op"),
    ("v_cndmask_b32", 7, "op"), ("v_fma_f64", 8, "op"), ("v_xor_b32", 9, "op"), ("v_lshl_add_u32", 10, "op"),
    ("CT butterfly, 31-bit p (2013265921)", 11, "bfly"), ("CT butterfly, lazy, p < 2^30 (998244353)", 12, "bfly"),
    ("GS butterfly, 31-bit p (2013265921)", 13, "bfly"), ("GS butterfly, lazy, p < 2^30 (998244353)", 14, "bfly"),
    ("v_mov_b32 DPP row_shr:1", 15, "op"), ("v_permlane32_swap_b32 (one per register pair)", 16, "op"),
    ("ds_bpermute_b32", 17, "op"),
]
PER_ITER_OF = {16: 64}     # the swap probe issues 64 instructions per thread and iteration
PER_ITER = 16 * 8          # operations (or butterflies) per thread and iteration
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
UNIT_PEAK = CUS * LANES * CLOCK_HZ  # one 32-bit VALU lane-op per lane per clock: 39.3 T/s


def _params(p: int, g: int):
    pinv = pow(p, -1, 1 << 32)
    w = pow(g, (p - 1) >> 16, p)
    ws = (w << 32) // p
    return p, pinv, w, ws


def measure(iters: int = 2000, grid: int = 8192, reps: int = 5):
    import torch
    lib = ctypes.CDLL(LIB_PATH)
    lib.valu_rate_launch.restype = ctypes.c_int
    lib.valu_rate_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    out = torch.empty(grid * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    rows = []
    for name, op, kind in PROBES:
        if op in (11, 13):
            p, pinv, w, ws = _params(2013265921, 31)
        else:
            p, pinv, w, ws = _params(998244353, 3)
        h = ctypes.c_void_p(stream.cuda_stream)

        def launch():
            rc = lib.valu_rate_launch(op, grid, iters, ctypes.c_void_p(out.data_ptr()), p, pinv, w, ws, h)
            if rc != 0:
                raise RuntimeError("valu_rate_launch(%s) returned %d" % (name, rc))

        with torch.cuda.stream(stream):
            for _ in range(2):
                launch()
            best = None
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                launch()
                e1.record(stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
        count = grid * 256 * iters * PER_ITER_OF.get(op, PER_ITER)
        rate = count / (best * 1e-3)
        rows.append({"probe": name, "kind": kind, "ms": best, "count": count, "rate": rate,
                     "per_cu_clock": rate / (CUS * CLOCK_HZ)})
        print("%-42s %9.3f ms  %8.2f T/s  %6.2f per CU and clock" % (name, best, rate / 1e12, rate / (CUS * CLOCK_HZ)),
              flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--grid", type=int, default=8192)
    ap.add_argument("--json", default="")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        sys.exit("valu_rates needs a GPU")
    print("device: %s, %d CUs; one lane-op per lane per clock at 2.4 GHz = %.2f T/s"
          % (torch.cuda.get_device_name(0), torch.cuda.get_device_properties(0).multi_processor_count,
             UNIT_PEAK / 1e12), flush=True)
    rows = measure(a.iters, a.grid)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
