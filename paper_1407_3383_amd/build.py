"""Build script for the HIP library (gfx950): hipcc -> libntt_mi355x.so in-tree.

Each translation unit is compiled to an object in parallel (no device code crosses
translation units), then linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libntt_mi355x.so")
SOURCES = ["host.cpp", "server.cpp", "kernels_poly.hip", "kernels_poly_w32.hip", "kernels_poly_w32c3.hip", "kernels_poly_w32c4.hip", "kernels_poly_w64.hip", "kernels_poly_f64.hip", "kernels_ntt.hip", "kernels_pass.hip", "kernels_split.hip", "kernels_crt.hip",
           "kernels_matrix.hip", "kernels_arith.hip", "kernels_tft.hip"]
# Issue-rate probes of the vector ALU (measurement only, a library of their own).
PROBE_SRC = "valu_rates.hip"
PROBE_LIB = os.path.join(HERE, "libvalu_rates.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", "-o", obj] + (["-x", "hip"] if src.endswith(".cpp") else []) + [path]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = False) -> str:
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-shared", "-o", tmp, os.path.join(CSRC, PROBE_SRC)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
