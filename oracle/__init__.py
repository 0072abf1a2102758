"""CPU oracle for the NTT / polynomial-product / integer-product path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg import this package.  It shares no code with the HIP
library (``paper_1407_3383_amd``) and imports nothing from it; the only common
module is the seeded input generator ``paper_1407_3383_amd.inputs``, which holds no
arithmetic of the method.

Contents
--------
* ``ntt_oracle.c`` (built into ``libntt_oracle.so`` with gcc): the plain definitions
  in C with unsigned __int128 products and ``%`` reductions -- DFT by definition,
  Horner evaluation, a textbook radix-2 transform, schoolbook and transform-based
  polynomial products, the schoolbook polynomial matrix product, schoolbook and
  three-prime integer products, Garner digits.
* ``numtheory``: primality (deterministic Miller-Rabin), primitive roots, roots of
  unity, the rule that picks the ~62-bit prime, Barrett / Shoup / Montgomery
  constants by their definitions -- in Python integers.
* ``algorithm1``: the paper's Algorithm 1 (section 5.1) and the TFT definition, in
  Python integers, for small sizes.
* ``modarith``: word-size-generic forms of the paper's Functions 2, 6, 8 and 13
  (section 2), for exhaustive checks of their propositions.

Every function states the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntt_oracle.c")
_LIB = os.path.join(_HERE, "libntt_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64, sz, vp = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p
        sig = {
            "orc_mulmod": (u64, [u64, u64, u64]),
            "orc_addmod": (u64, [u64, u64, u64]),
            "orc_submod": (u64, [u64, u64, u64]),
            "orc_powmod": (u64, [u64, u64, u64]),
            "orc_invmod": (u64, [u64, u64]),
            "orc_bitrev": (sz, [sz, ctypes.c_uint]),
            "orc_dft": (None, [u64, u64, vp, vp, sz]),
            "orc_horner": (u64, [u64, vp, sz, u64]),
            "orc_horner_many": (None, [u64, vp, sz, vp, vp, sz]),
            "orc_ntt": (None, [u64, u64, vp, sz]),
            "orc_intt": (None, [u64, u64, vp, sz]),
            "orc_polymul_schoolbook": (None, [u64, vp, sz, vp, sz, vp]),
            "orc_polymul_ntt": (ctypes.c_int, [u64, u64, sz, vp, sz, vp, sz, vp]),
            "orc_intmul_schoolbook": (None, [vp, sz, vp, sz, vp]),
            "orc_intmul_3prime": (ctypes.c_int, [vp, sz, vp, sz, vp, vp, vp, sz]),
            "orc_garner_digits": (None, [vp, vp, vp, sz, vp, vp, vp, vp]),
            "orc_mulmod_vec": (None, [u64, vp, vp, vp, sz]),
            "orc_limbs32_mod": (u64, [vp, sz, u64]),
            "orc_limbs16_mod": (u64, [vp, sz, u64]),
            "orc_polymatmul": (None, [u64, sz, vp, vp, sz, vp]),
            "orc_polymatmul_coeff": (u64, [u64, sz, vp, vp, sz, sz, sz, sz]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------- scalar

def mulmod(a: int, b: int, p: int) -> int:
    return int(lib().orc_mulmod(a, b, p))


def powmod(a: int, e: int, p: int) -> int:
    return int(lib().orc_powmod(a, e, p))


def invmod(a: int, p: int) -> int:
    return int(lib().orc_invmod(a, p))


def bitrev(i: int, k: int) -> int:
    """The bitwise mirror [i]_k of section 5.1."""
    return int(lib().orc_bitrev(i, k))


def bitrev_perm(k: int) -> np.ndarray:
    """Index vector r with r[i] = [i]_k."""
    i = np.arange(1 << k, dtype=np.int64)
    r = np.zeros_like(i)
    for b in range(k):
        r |= ((i >> b) & 1) << (k - 1 - b)
    return r


# ----------------------------------------------------------------------------- transforms

def dft(a, p: int, w: int) -> np.ndarray:
    """FFT by definition (section 5.1): out_i = sum_j w^(ij) a_j.  O(n^2)."""
    x = _u64(a)
    out = np.empty_like(x)
    lib().orc_dft(p, w, _ptr(x), _ptr(out), x.size)
    return out


def ntt(a, p: int, w: int) -> np.ndarray:
    """Textbook radix-2 transform, natural order in and out (same result as ``dft``)."""
    x = _u64(a).copy()
    lib().orc_ntt(p, w, _ptr(x), x.size)
    return x


def intt(a, p: int, w: int) -> np.ndarray:
    """Inverse transform including the factor n^-1, so intt(ntt(a)) = a."""
    x = _u64(a).copy()
    lib().orc_intt(p, w, _ptr(x), x.size)
    return x


def tft_order(a_hat: np.ndarray) -> np.ndarray:
    """Reorder a natural-order transform into the TFT order of section 5.1:
    position i holds a_hat[[i]_k]."""
    n = a_hat.size
    k = n.bit_length() - 1
    return a_hat[bitrev_perm(k)]


def tft(a, n: int, l_out: int, p: int, w: int) -> np.ndarray:
    """TFT_w of section 5.1 for a transform length n: the input (len(a) <= n
    coefficients, zero beyond) transformed by the textbook transform, reordered into
    the TFT order, and its first l_out values kept."""
    x = np.zeros(n, dtype=np.uint64)
    v = _u64(a)
    x[:v.size] = v
    return tft_order(ntt(x, p, w))[:l_out].copy()


def horner(a, p: int, x: int) -> int:
    """A(x) = sum_j a_j x^j (section 5.1: a_hat_i = A(w^i))."""
    v = _u64(a)
    return int(lib().orc_horner(p, _ptr(v), v.size, x))


def horner_many(a, p: int, xs) -> np.ndarray:
    v = _u64(a)
    xv = _u64(xs)
    out = np.empty_like(xv)
    lib().orc_horner_many(p, _ptr(v), v.size, _ptr(xv), _ptr(out), xv.size)
    return out


# ----------------------------------------------------------------------------- products

def polymul_schoolbook(a, b, p: int) -> np.ndarray:
    """c_k = sum_{i+j=k} a_i b_j mod p, k < la + lb - 1 (section 5.2's product)."""
    x, y = _u64(a), _u64(b)
    if x.size == 0 or y.size == 0:
        return np.zeros(0, dtype=np.uint64)
    c = np.empty(x.size + y.size - 1, dtype=np.uint64)
    lib().orc_polymul_schoolbook(p, _ptr(x), x.size, _ptr(y), y.size, _ptr(c))
    return c


def polymul_ntt(a, b, p: int, g: int | None = None) -> np.ndarray:
    """Zero-padded transform product (section 5.2) with the oracle's textbook transform."""
    from . import numtheory
    x, y = _u64(a), _u64(b)
    if x.size == 0 or y.size == 0:
        return np.zeros(0, dtype=np.uint64)
    lc = x.size + y.size - 1
    n = 1 << max(0, (lc - 1).bit_length())
    w = numtheory.root_of_unity(p, n, g)
    c = np.empty(lc, dtype=np.uint64)
    rc = lib().orc_polymul_ntt(p, w, n, _ptr(x), x.size, _ptr(y), y.size, _ptr(c))
    if rc != 0:
        raise RuntimeError("orc_polymul_ntt failed: %d" % rc)
    return c


def _matrix_operands(A, B):
    x, y = np.asarray(A), np.asarray(B)
    if x.ndim != 3 or x.shape != y.shape or x.shape[0] != x.shape[1]:
        raise ValueError("A and B must both have shape (n, n, d)")
    return _u64(x.reshape(-1)), _u64(y.reshape(-1)), x.shape[0], x.shape[2]


def polymatmul(A, B, p: int) -> np.ndarray:
    """Polynomial matrix product (section 5.2): A, B of shape (n, n, d) over F_p,
    C[i, j] = sum_l A[i, l] * B[l, j] as polynomials, shape (n, n, 2d - 1)."""
    x, y, n, d = _matrix_operands(A, B)
    if n == 0 or d == 0:
        return np.zeros((n, n, max(2 * d - 1, 0)), dtype=np.uint64)
    c = np.empty(n * n * (2 * d - 1), dtype=np.uint64)
    lib().orc_polymatmul(p, n, _ptr(x), _ptr(y), d, _ptr(c))
    return c.reshape(n, n, 2 * d - 1)


def polymatmul_coeff(A, B, p: int, i: int, j: int, k: int) -> int:
    """One coefficient C[i, j][k] of the polynomial matrix product, O(n d)."""
    x, y, n, d = _matrix_operands(A, B)
    return int(lib().orc_polymatmul_coeff(p, n, _ptr(x), _ptr(y), d, i, j, k))


INTMUL_PRIMES = (998244353, 469762049, 167772161)
INTMUL_ROOTS = (3, 3, 3)


def intmul_schoolbook(a16, b16) -> np.ndarray:
    """Exact product of little-endian 16-bit-limb integers, as ceil((na+nb)/2) 32-bit limbs."""
    a = np.ascontiguousarray(np.asarray(a16, dtype=np.uint16))
    b = np.ascontiguousarray(np.asarray(b16, dtype=np.uint16))
    c = np.zeros((a.size + b.size + 1) // 2, dtype=np.uint32)
    lib().orc_intmul_schoolbook(_ptr(a), a.size, _ptr(b), b.size, _ptr(c))
    return c


def intmul_3prime(a16, b16, primes=INTMUL_PRIMES, gens=INTMUL_ROOTS) -> np.ndarray:
    """Kronecker segmentation (h = 16) + three-prime transform + Garner + carry (section 5.3)."""
    from . import numtheory
    a = np.ascontiguousarray(np.asarray(a16, dtype=np.uint16))
    b = np.ascontiguousarray(np.asarray(b16, dtype=np.uint16))
    c = np.zeros((a.size + b.size + 1) // 2, dtype=np.uint32)
    if a.size == 0 or b.size == 0:
        return c
    lc = a.size + b.size - 1
    n = 1 << max(0, (lc - 1).bit_length())
    pr = _u64(primes)
    roots = _u64([numtheory.root_of_unity(int(q), n, int(g)) for q, g in zip(primes, gens)])
    rc = lib().orc_intmul_3prime(_ptr(a), a.size, _ptr(b), b.size, _ptr(c), _ptr(pr), _ptr(roots), n)
    if rc != 0:
        raise RuntimeError("orc_intmul_3prime failed: %d" % rc)
    return c


def intmul_pyint(a16, b16) -> np.ndarray:
    """Exact product with Python's arbitrary-precision integers."""
    a = np.ascontiguousarray(np.asarray(a16, dtype="<u2"))
    b = np.ascontiguousarray(np.asarray(b16, dtype="<u2"))
    nc32 = (a.size + b.size + 1) // 2
    A = int.from_bytes(a.tobytes(), "little")
    B = int.from_bytes(b.tobytes(), "little")
    return np.frombuffer((A * B).to_bytes(4 * nc32, "little"), dtype="<u4").astype(np.uint32)


def _int_of_limbs32(x) -> int:
    return int.from_bytes(np.ascontiguousarray(np.asarray(x, dtype="<u4")).tobytes(), "little")


def intmatmul_entry_pyint(A32, B32, i: int, j: int) -> int:
    """Entry (i, j) of the integer matrix product (section 5.3) as a Python integer:
    sum over l of A[i, l] B[l, j], each entry a little-endian 32-bit limb vector."""
    n = A32.shape[0]
    return sum(_int_of_limbs32(A32[i, l]) * _int_of_limbs32(B32[l, j]) for l in range(n))


def intmatmul_pyint(A32, B32) -> np.ndarray:
    """Integer matrix product (section 5.3): A, B of shape (n, n, na) 32-bit limbs ->
    C of shape (n, n, 2 na + 1) limbs, exactly, with Python's integers."""
    n, na = A32.shape[0], A32.shape[2]
    out = np.zeros((n, n, 2 * na + 1), dtype=np.uint32)
    for i in range(n):
        for j in range(n):
            v = intmatmul_entry_pyint(A32, B32, i, j)
            out[i, j] = np.frombuffer(v.to_bytes(4 * (2 * na + 1), "little"), dtype="<u4")
    return out


def garner_digits(r1, r2, r3, primes=INTMUL_PRIMES):
    """Garner's mixed-radix digits (x1, x2, x3) of each residue triple."""
    v1, v2, v3 = _u64(r1), _u64(r2), _u64(r3)
    n = v1.size
    pr = _u64(primes)
    x1, x2, x3 = (np.empty(n, dtype=np.uint64) for _ in range(3))
    lib().orc_garner_digits(_ptr(v1), _ptr(v2), _ptr(v3), n, _ptr(pr), _ptr(x1), _ptr(x2), _ptr(x3))
    return x1, x2, x3


def limbs32_mod(x, q: int) -> int:
    v = np.ascontiguousarray(np.asarray(x, dtype=np.uint32))
    return int(lib().orc_limbs32_mod(_ptr(v), v.size, q))


def limbs16_mod(x, q: int) -> int:
    v = np.ascontiguousarray(np.asarray(x, dtype=np.uint16))
    return int(lib().orc_limbs16_mod(_ptr(v), v.size, q))
