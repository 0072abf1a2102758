"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This module holds no modular arithmetic: it only draws uniform residues, 16-bit
integer limbs and a few structured vectors from numpy's PCG64 generator, seeded by
``SeedSequence([14073383, config_id, item])`` so that any single item of a batch can
be regenerated on its own.

The workloads mirror the paper's own timing runs (section 5: FFTs, polynomial and
integer products on uniformly random data); there is no public dataset involved.
"""
from __future__ import annotations

import numpy as np

SEED = 14073383

# Workload identifiers (the ``config_id`` component of the seed).
CFG_POLYMUL_8K = 0        # one polymul mod 998244353, two length-4096 operands
CFG_POLYMUL_BATCH = 1     # 1024 polymuls mod 2013265921, length 2^15 operands
CFG_NTT_2_24 = 2          # one length-2^24 transform mod 469762049
CFG_INTMUL = 3            # 2^21 x 2^21 16-bit-limb integer product
CFG_SERVE = 4             # serving mix
CFG_FFT = 5               # transforms of length 2^8..2^20, 2^24 words per call
CFG_TEST = 99             # ad-hoc test inputs

P_998 = 998244353         # 119 * 2^23 + 1
P_2013 = 2013265921       # 15 * 2^27 + 1
P_469 = 469762049         # 7 * 2^26 + 1
P_167 = 167772161         # 5 * 2^25 + 1


def rng(config_id: int, item: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, config_id, item])))


def residue_dtype(p: int):
    return np.uint32 if p < (1 << 32) else np.uint64


def residues(p: int, n: int, config_id: int, item: int = 0, stream: int = 0) -> np.ndarray:
    """n residues uniform in [0, p), uint32 when p < 2^32 else uint64."""
    g = rng(config_id, item * 4 + stream)
    return g.integers(0, p, size=n, dtype=np.uint64).astype(residue_dtype(p))


def limbs16(n: int, config_id: int, item: int = 0, stream: int = 0, top_nonzero: bool = True) -> np.ndarray:
    """n little-endian 16-bit limbs, uniform; the top limb drawn from [1, 2^16) when asked."""
    g = rng(config_id, item * 4 + stream)
    x = g.integers(0, 1 << 16, size=n, dtype=np.uint32).astype(np.uint16)
    if top_nonzero and n > 0:
        x[-1] = np.uint16(g.integers(1, 1 << 16))
    return x


def limbs32(n: int, config_id: int, item: int = 0, stream: int = 0) -> np.ndarray:
    """n little-endian 32-bit limbs, uniform in [0, 2^32)."""
    g = rng(config_id, item * 4 + stream)
    return g.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)


def polymul_8k_inputs():
    """Two length-4096 operands mod 998244353."""
    p = P_998
    return p, residues(p, 4096, CFG_POLYMUL_8K, 0, 0), residues(p, 4096, CFG_POLYMUL_8K, 0, 1)


def polymul_batch_item(item: int, length: int = 1 << 15, p: int = P_2013):
    return residues(p, length, CFG_POLYMUL_BATCH, item, 0), residues(p, length, CFG_POLYMUL_BATCH, item, 1)


def polymul_batch_inputs(items: int = 1024, length: int = 1 << 15, p: int = P_2013):
    """Row-major [item][coefficient] operand matrices."""
    a = np.empty((items, length), dtype=residue_dtype(p))
    b = np.empty((items, length), dtype=residue_dtype(p))
    for i in range(items):
        a[i], b[i] = polymul_batch_item(i, length, p)
    return p, a, b


def ntt_2_24_inputs(log2n: int = 24, p: int = P_469):
    return p, residues(p, 1 << log2n, CFG_NTT_2_24, 0, 0)


def intmul_inputs(nlimbs: int = 1 << 21, config_id: int = CFG_INTMUL, item: int = 0):
    return limbs16(nlimbs, config_id, item, 0), limbs16(nlimbs, config_id, item, 1)


def structured(kind: str, p: int, n: int, j: int = 0) -> np.ndarray:
    """Edge-case vectors: zeros, all p-1, delta_j, alternating 0/p-1, ones."""
    dt = residue_dtype(p)
    if kind == "zeros":
        return np.zeros(n, dtype=dt)
    if kind == "pm1":
        return np.full(n, p - 1, dtype=dt)
    if kind == "ones":
        return np.ones(n, dtype=dt)
    if kind == "delta":
        x = np.zeros(n, dtype=dt)
        x[j] = 1
        return x
    if kind == "alternating":
        x = np.zeros(n, dtype=dt)
        x[1::2] = p - 1
        return x
    raise ValueError(kind)


def serve_requests(count: int, primes, lo_log2: float = 8.0, hi_log2: float = 20.0, seed_item: int = 0):
    """Request mix: length L = floor(2^U(lo, hi)), prime uniform over ``primes``.

    Returns a list of (prime, L, request_id); operands come from ``serve_operands`` so
    that a single request can be replayed alone and nothing large is held up front.
    """
    g = rng(CFG_SERVE, seed_item)
    out = []
    for r in range(count):
        L = int(np.floor(2.0 ** g.uniform(lo_log2, hi_log2)))
        p = int(primes[int(g.integers(0, len(primes)))])
        out.append((p, L, 1 + r + seed_item * 10_000_000))
    return out


def serve_operands(p: int, L: int, request_id: int):
    return residues(p, L, CFG_SERVE, request_id, 0), residues(p, L, CFG_SERVE, request_id, 1)


def poisson_arrivals(count: int, rate_per_s: float, seed_item: int = 0) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream."""
    g = rng(CFG_SERVE, 1_000_000 + seed_item)
    return np.cumsum(g.exponential(1.0 / rate_per_s, size=count))
