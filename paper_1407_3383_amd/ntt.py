"""ctypes binding of libntt_mi355x.so (the C ABI in include/ntt_mi355x.h).

Argument marshalling only: every step of the computation runs in the HIP kernels of
the library.  PyTorch provides device memory (tensors) and streams.  Residue vectors
are passed as int32 tensors (uint32 residues, p < 2^31) or int64 tensors (uint64
residues, 2^31 <= p < 2^62) holding the residues' bit patterns; limbs of the integer
product are int16 (in) and int32 (out) tensors.  Use ``to_device`` / ``to_numpy`` to
move numpy unsigned arrays in and out.

There is no fallback: if the library is missing or no GPU is visible the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libntt_mi355x.so")
# Launch-shape choices written by the autotuner for this GPU; loaded with the library.
# NTT_TUNE_FILE names another file, or (empty) none.
TUNE_FILE = os.path.join(_HERE, "tuning", "gfx950.txt")

NTT_ARITH_SHOUP, NTT_ARITH_MONT, NTT_ARITH_RED1, NTT_ARITH_RED2, NTT_ARITH_CT, NTT_ARITH_GS = range(6)
NTT_OK = 0
NTT_EINVAL = -1
NTT_ENOTPRIME = -2
NTT_ENOROOT = -3
NTT_ERANGE = -4
NTT_ENOMEM = -5
NTT_EDEVICE = -6
NTT_EUNSUPPORTED = -7

NTT_BITREV_OUT = 1
NTT_BITREV_IN = 2
NTT_VALIDATE = 4
NTT_FP64 = 8

# Every symbol the header declares.
EXPORTS = (
    "ntt_strerror", "ntt_last_error", "ntt_is_prime", "ntt_smallest_generator", "ntt_find_prime",
    "ntt_plan_create", "ntt_plan_destroy", "ntt_plan_get_info", "ntt_workspace_bytes",
    "ntt_forward", "ntt_inverse", "polymul_workspace_bytes", "polymul_modp",
    "polymul_batch_workspace_bytes", "polymul_modp_batch", "polymul_batch_create",
    "polymul_batch_launch_workspace_bytes", "polymul_batch_launch", "polymul_batch_destroy",
    "intmul_workspace_bytes", "intmul_crt", "intmul_chunk_bits", "intmul32_workspace_bytes", "intmul_crt32",
    "polymatmul_workspace_bytes", "polymatmul_modp", "polymul_f64_batch_workspace_bytes", "polymul_f64_batch",
    "polymul_f64_batch_create", "intmatmul32_workspace_bytes", "intmatmul_crt32", "ntt_arith_apply",
    "ntt_tune_set", "ntt_tune_get", "ntt_tune_clear", "ntt_tune_load", "ntt_plan_cache_clear",
    "ntt_graph_begin", "ntt_graph_end", "ntt_graph_launch", "ntt_graph_destroy",
    "ntt_server_create", "ntt_server_submit", "ntt_server_progress", "ntt_server_stats", "ntt_server_destroy",
    "polymul_modp_noalloc", "ntt_tft_workspace_bytes", "ntt_tft_forward", "ntt_tft_inverse",
)


class NTTError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed: %s (%d)%s" % (where, _strerror(code), code, (": " + detail) if detail else ""))
        self.code = code


class PolymulDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("a", ctypes.c_void_p), ("la", ctypes.c_size_t),
                ("b", ctypes.c_void_p), ("lb", ctypes.c_size_t), ("c", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("g", ctypes.c_uint64), ("w", ctypes.c_uint64),
                ("w_inv", ctypes.c_uint64), ("n_inv", ctypes.c_uint64), ("log2n", ctypes.c_uint32),
                ("word_bits", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("passes", ctypes.c_uint32),
                ("row_log2", ctypes.c_uint32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libntt_mi355x.so is not built (run __graft_entry__.build())")
    # torch first: its bundled HIP runtime (same soname) must be the one the library
    # binds to, so that torch's streams and allocations are valid handles for it.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    u64, sz, vp, u32, ci = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
    sig = {
        "ntt_strerror": (ctypes.c_char_p, [ci]),
        "ntt_last_error": (ctypes.c_char_p, []),
        "ntt_is_prime": (ci, [u64]),
        "ntt_smallest_generator": (u64, [u64]),
        "ntt_find_prime": (u64, [u32, u32]),
        "ntt_plan_create": (ci, [ctypes.POINTER(vp), u64, u64, u32, u32, vp]),
        "ntt_plan_destroy": (ci, [vp]),
        "ntt_plan_get_info": (ci, [vp, ctypes.POINTER(PlanInfo)]),
        "ntt_workspace_bytes": (sz, [vp, sz]),
        "ntt_forward": (ci, [vp, vp, vp, sz, sz, vp, sz, vp]),
        "ntt_inverse": (ci, [vp, vp, vp, sz, sz, vp, sz, vp]),
        "ntt_tft_workspace_bytes": (sz, [vp, sz]),
        "ntt_tft_forward": (ci, [vp, vp, sz, vp, sz, sz, sz, sz, vp, sz, vp]),
        "ntt_tft_inverse": (ci, [vp, vp, vp, sz, sz, sz, sz, vp, sz, vp]),
        "polymul_workspace_bytes": (sz, [u64, sz, sz]),
        "polymul_modp": (ci, [u64, vp, sz, vp, sz, vp, vp, sz, vp]),
        "polymul_modp_noalloc": (ci, [u64, vp, sz, vp, sz, vp, vp]),
        "polymul_batch_workspace_bytes": (sz, [ctypes.POINTER(PolymulDesc), sz]),
        "polymul_modp_batch": (ci, [ctypes.POINTER(PolymulDesc), sz, vp, sz, vp]),
        "polymul_batch_create": (ci, [ctypes.POINTER(vp), ctypes.POINTER(PolymulDesc), sz]),
        "polymul_batch_launch_workspace_bytes": (sz, [vp]),
        "polymul_batch_launch": (ci, [vp, vp, sz, vp]),
        "polymul_batch_destroy": (ci, [vp]),
        "intmul_workspace_bytes": (sz, [sz, sz]),
        "intmul_crt": (ci, [vp, sz, vp, sz, vp, vp, sz, vp]),
        "intmul_chunk_bits": (ci, [sz, sz]),
        "intmul32_workspace_bytes": (sz, [sz, sz]),
        "intmul_crt32": (ci, [vp, sz, vp, sz, vp, vp, sz, vp]),
        "polymatmul_workspace_bytes": (sz, [u64, sz, sz]),
        "polymatmul_modp": (ci, [u64, sz, vp, vp, sz, vp, vp, sz, vp]),
        "polymul_f64_batch_workspace_bytes": (sz, [ctypes.POINTER(PolymulDesc), sz]),
        "polymul_f64_batch": (ci, [ctypes.POINTER(PolymulDesc), sz, vp, sz, vp]),
        "polymul_f64_batch_create": (ci, [ctypes.POINTER(vp), ctypes.POINTER(PolymulDesc), sz]),
        "intmatmul32_workspace_bytes": (sz, [sz, sz]),
        "intmatmul_crt32": (ci, [sz, vp, vp, sz, vp, vp, sz, vp]),
        "ntt_arith_apply": (ci, [ctypes.c_int, ctypes.c_int, u64, vp, vp, vp, u64, u64, vp, sz, vp]),
        "ntt_tune_set": (ci, [ctypes.c_char_p, ctypes.c_int64]),
        "ntt_tune_get": (ci, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]),
        "ntt_tune_clear": (ci, []),
        "ntt_tune_load": (ci, [ctypes.c_char_p]),
        "ntt_plan_cache_clear": (ci, []),
        "ntt_server_create": (ci, [ctypes.POINTER(vp), sz, ci, sz]),
        "ntt_server_submit": (ci, [vp, u64, ci, u64, vp, sz, vp, sz, vp]),
        "ntt_server_progress": (ci, [vp, ctypes.POINTER(u64), sz, ctypes.POINTER(sz)]),
        "ntt_server_stats": (ci, [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "ntt_server_destroy": (ci, [vp]),
        "ntt_graph_begin": (ci, [vp]),
        "ntt_graph_end": (ci, [vp, ctypes.POINTER(vp)]),
        "ntt_graph_launch": (ci, [vp, vp]),
        "ntt_graph_destroy": (ci, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    tune_file = os.environ.get("NTT_TUNE_FILE", TUNE_FILE)
    if tune_file and os.path.exists(tune_file):
        rc = L.ntt_tune_load(tune_file.encode())
        if rc != NTT_OK:
            raise NTTError(rc, "ntt_tune_load", L.ntt_last_error().decode())
    _lib = L
    return L


def _strerror(code: int) -> str:
    try:
        return load().ntt_strerror(code).decode()
    except Exception:
        return "error"


def _check(rc: int, where: str):
    if rc != NTT_OK:
        raise NTTError(rc, where, load().ntt_last_error().decode())


# ----------------------------------------------------------------------------- host helpers

def is_prime(n: int) -> bool:
    return bool(load().ntt_is_prime(n))


def smallest_generator(p: int) -> int:
    return int(load().ntt_smallest_generator(p))


def find_prime(bits: int, l: int) -> int:
    return int(load().ntt_find_prime(bits, l))


def word_bits(p: int) -> int:
    return 32 if p < (1 << 31) else 64


def tune_set(key: str, value: int):
    _check(load().ntt_tune_set(key.encode(), value), "ntt_tune_set")


def tune_get(key: str) -> Optional[int]:
    v = ctypes.c_int64()
    return int(v.value) if load().ntt_tune_get(key.encode(), ctypes.byref(v)) == NTT_OK else None


def tune_clear():
    _check(load().ntt_tune_clear(), "ntt_tune_clear")


def tune_load(path: str):
    _check(load().ntt_tune_load(path.encode()), "ntt_tune_load")


def plan_cache_clear():
    _check(load().ntt_plan_cache_clear(), "ntt_plan_cache_clear")


# ----------------------------------------------------------------------------- tensors

def _torch():
    import torch
    return torch


def to_device(x: np.ndarray, device="cuda"):
    """numpy uint16/uint32/uint64 -> device tensor of the same bit pattern."""
    torch = _torch()
    x = np.ascontiguousarray(x)
    view = {np.dtype(np.uint16): np.int16, np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}
    if x.dtype in view:
        x = x.view(view[x.dtype])
    return torch.from_numpy(x).to(device)


def to_numpy(t, unsigned=True) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if not unsigned:
        return a
    view = {np.dtype(np.int16): np.uint16, np.dtype(np.int32): np.uint32, np.dtype(np.int64): np.uint64}
    return a.view(view[a.dtype]) if a.dtype in view else a


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _workspace(nbytes: int, device):
    if nbytes == 0:
        return None
    torch = _torch()
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _res_dtype(p: int):
    torch = _torch()
    return torch.int32 if word_bits(p) == 32 else torch.int64


# ----------------------------------------------------------------------------- products

def polymul(a, b, p: int, out=None, stream=None, workspace=None):
    """c = a * b mod p (linear product, len(a) + len(b) - 1 coefficients)."""
    torch = _torch()
    L = load()
    la, lb = a.numel(), b.numel()
    lc = la + lb - 1 if la and lb else 0
    if out is None:
        out = torch.empty(lc, dtype=_res_dtype(p), device=a.device)
    need = L.polymul_workspace_bytes(p, la, lb)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, a.device)
    _check(L.polymul_modp(p, _ptr(a), la, _ptr(b), lb, _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                          _stream(stream)), "polymul_modp")
    return out


def polymul_noalloc(a, b, p: int, out, stream=None):
    """polymul_modp_noalloc: c = a * b mod p into the caller's `out` (la + lb - 1
    coefficients), scratch in the library's fixed device array; the plan of (p, N)
    must already exist (an earlier polymul call with the same p and length)."""
    _check(load().polymul_modp_noalloc(p, _ptr(a), a.numel(), _ptr(b), b.numel(), _ptr(out), _stream(stream)),
           "polymul_modp_noalloc")
    return out


def polymul_batch(pairs: Sequence, primes: Sequence[int], outs=None, stream=None, workspace=None):
    """Products of many (a, b) pairs, one prime each, in one batched call."""
    torch = _torch()
    L = load()
    n = len(pairs)
    if outs is None:
        outs = []
        for (a, b), p in zip(pairs, primes):
            lc = a.numel() + b.numel() - 1 if a.numel() and b.numel() else 0
            outs.append(torch.empty(lc, dtype=_res_dtype(p), device=a.device))
    descs = (PolymulDesc * max(n, 1))()
    for i, ((a, b), p) in enumerate(zip(pairs, primes)):
        descs[i] = PolymulDesc(p, _ptr(a).value, a.numel(), _ptr(b).value, b.numel(), _ptr(outs[i]).value)
    need = L.polymul_batch_workspace_bytes(descs, n)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, pairs[0][0].device if n else "cuda")
    _check(L.polymul_modp_batch(descs, n, _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)),
           "polymul_modp_batch")
    return outs


def polymul_f64_rows(A, B, p: int, out=None, stream=None, workspace=None, descs=None):
    """Row-wise products of two [items, L] float64 matrices of residues mod p < 2^49,
    computed in FP64 arithmetic (polymul_f64_batch); out is [items, la + lb - 1] float64."""
    torch = _torch()
    items, la = A.shape
    lb = B.shape[1]
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise ValueError("operands must be float64 residues")
    if out is None:
        out = torch.empty((items, la + lb - 1), dtype=torch.float64, device=A.device)
    L = load()
    if descs is None:
        descs = f64_row_descs(A, B, out, p)
    need = L.polymul_f64_batch_workspace_bytes(descs, items)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, A.device)
    _check(L.polymul_f64_batch(descs, items, _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)),
           "polymul_f64_batch")
    return out


def f64_row_descs(A, B, out, p: int):
    items, la = A.shape
    lb = B.shape[1]
    descs = (PolymulDesc * items)()
    a0, b0, c0 = A.data_ptr(), B.data_ptr(), out.data_ptr()
    for i in range(items):
        descs[i] = PolymulDesc(p, a0 + 8 * la * i, la, b0 + 8 * lb * i, lb, c0 + 8 * out.shape[1] * i)
    return descs


def polymul_rows(A, B, p: int, out=None, stream=None, workspace=None):
    """Row-wise products of two [items, L] matrices (one batched launch)."""
    torch = _torch()
    items, la = A.shape
    lb = B.shape[1]
    if out is None:
        out = torch.empty((items, la + lb - 1), dtype=_res_dtype(p), device=A.device)
    L = load()
    descs = (PolymulDesc * items)()
    a0, b0, c0 = A.data_ptr(), B.data_ptr(), out.data_ptr()
    esz = A.element_size()
    sa, sb, sc = A.stride(0) * esz, B.stride(0) * esz, out.stride(0) * esz
    for i in range(items):
        descs[i] = PolymulDesc(p, a0 + i * sa, la, b0 + i * sb, lb, c0 + i * sc)
    need = L.polymul_batch_workspace_bytes(descs, items)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, A.device)
    _check(L.polymul_modp_batch(descs, items, _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)),
           "polymul_modp_batch")
    return out


class Batch:
    """Reusable batch handle (polymul_batch_create): descriptors live on the device;
    each call only launches kernels, so it can be repeated or graph-captured."""

    def __init__(self, pairs_or_descs, primes=None, outs=None, f64=False):
        """f64: operands and outputs are float64 residues (polymul_f64_batch_create)."""
        L = load()
        if primes is not None:
            descs = (PolymulDesc * max(len(pairs_or_descs), 1))()
            for i, ((a, b), p) in enumerate(zip(pairs_or_descs, primes)):
                descs[i] = PolymulDesc(p, _ptr(a).value, a.numel(), _ptr(b).value, b.numel(), _ptr(outs[i]).value)
            count = len(pairs_or_descs)
            self._keep = (pairs_or_descs, outs)
        else:
            descs, count = pairs_or_descs
        h = ctypes.c_void_p()
        if f64:
            _check(L.polymul_f64_batch_create(ctypes.byref(h), descs, count), "polymul_f64_batch_create")
        else:
            _check(L.polymul_batch_create(ctypes.byref(h), descs, count), "polymul_batch_create")
        self.handle = h
        self.count = count
        self.ws_bytes = int(L.polymul_batch_launch_workspace_bytes(h))
        self.ws = None

    @classmethod
    def rows(cls, A, B, out, p: int, f64: bool = False):
        """Row-wise products of [items, L] matrices into out[items, La + Lb - 1]."""
        items, la = A.shape
        lb = B.shape[1]
        descs = (PolymulDesc * items)()
        esz = A.element_size()
        for i in range(items):
            descs[i] = PolymulDesc(p, A.data_ptr() + i * A.stride(0) * esz, la,
                                   B.data_ptr() + i * B.stride(0) * esz, lb,
                                   out.data_ptr() + i * out.stride(0) * esz)
        self = cls((descs, items), f64=f64)
        self._keep = (A, B, out)
        if self.ws_bytes:
            self.ws = _workspace(self.ws_bytes, A.device)
        return self

    def __call__(self, stream=None, workspace=None):
        ws = workspace if workspace is not None else self.ws
        if self.ws_bytes and ws is None:
            import torch
            self.ws = ws = _workspace(self.ws_bytes, torch.device("cuda"))
        _check(load().polymul_batch_launch(self.handle, _ptr(ws), ws.numel() if ws is not None else 0,
                                           _stream(stream)), "polymul_batch_launch")

    def close(self):
        if getattr(self, "handle", None):
            load().polymul_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def intmul(a16, b16, out=None, stream=None, workspace=None):
    """Product of two little-endian 16-bit-limb integers -> ceil((na+nb)/2) 32-bit limbs."""
    torch = _torch()
    L = load()
    na, nb = a16.numel(), b16.numel()
    nc = (na + nb + 1) // 2
    if out is None:
        out = torch.empty(nc, dtype=torch.int32, device=a16.device)
    need = L.intmul_workspace_bytes(na, nb)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, a16.device)
    _check(L.intmul_crt(_ptr(a16), na, _ptr(b16), nb, _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                        _stream(stream)), "intmul_crt")
    return out


def intmul32(a32, b32, out=None, stream=None, workspace=None):
    """Product of two little-endian 32-bit-chunk integers -> na + nb 32-bit limbs."""
    torch = _torch()
    L = load()
    na, nb = a32.numel(), b32.numel()
    if out is None:
        out = torch.empty(na + nb, dtype=torch.int32, device=a32.device)
    need = L.intmul32_workspace_bytes(na, nb)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, a32.device)
    _check(L.intmul_crt32(_ptr(a32), na, _ptr(b32), nb, _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                          _stream(stream)), "intmul_crt32")
    return out


def polymatmul(A, B, p: int, out=None, stream=None, workspace=None):
    """Polynomial matrix product (section 5.2): A, B device tensors of shape (n, n, d)
    holding residues mod p < 2^31 (int32 bit patterns) -> C of shape (n, n, 2d - 1)."""
    torch = _torch()
    L = load()
    if A.dim() != 3 or A.shape != B.shape or A.shape[0] != A.shape[1]:
        raise ValueError("A and B must both have shape (n, n, d)")
    n, d = int(A.shape[0]), int(A.shape[2])
    if not (A.is_contiguous() and B.is_contiguous()):
        raise ValueError("A and B must be contiguous")
    lc = max(2 * d - 1, 0)
    if out is None:
        out = torch.empty((n, n, lc), dtype=torch.int32, device=A.device)
    need = L.polymatmul_workspace_bytes(p, n, d)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, A.device)
    _check(L.polymatmul_modp(p, n, _ptr(A), _ptr(B), d, _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                             _stream(stream)), "polymatmul_modp")
    return out


def intmatmul32(A, B, out=None, stream=None, workspace=None):
    """Integer matrix product (section 5.3): A, B device int32 tensors of shape
    (n, n, na) holding little-endian 32-bit limbs -> C of shape (n, n, 2 na + 1)."""
    torch = _torch()
    L = load()
    if A.dim() != 3 or A.shape != B.shape or A.shape[0] != A.shape[1]:
        raise ValueError("A and B must both have shape (n, n, na)")
    n, na = int(A.shape[0]), int(A.shape[2])
    if out is None:
        out = torch.empty((n, n, 2 * na + 1), dtype=torch.int32, device=A.device)
    need = L.intmatmul32_workspace_bytes(n, na)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, A.device)
    _check(L.intmatmul_crt32(n, _ptr(A), _ptr(B), na, _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                             _stream(stream)), "intmatmul_crt32")
    return out


def intmul_chunk_bits(na16: int, nb16: int) -> int:
    return int(load().intmul_chunk_bits(na16, nb16))


# ----------------------------------------------------------------------------- graphs

class Graph:
    """Records the library calls made on `stream` inside a `with` block as one HIP
    graph (ntt_graph_begin / ntt_graph_end); `replay()` reruns them.  Allocate every
    output and workspace before the block, and run each call once before recording
    it so that its plans exist."""

    def __init__(self, stream):
        self.stream = stream
        self.handle = None

    def __enter__(self):
        _check(load().ntt_graph_begin(_stream(self.stream)), "ntt_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        rc = load().ntt_graph_end(_stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            _check(rc, "ntt_graph_end")
        self.handle = h if rc == NTT_OK else None
        return False

    def replay(self, stream=None):
        if self.handle is None:
            raise RuntimeError("graph was not recorded")
        _check(load().ntt_graph_launch(self.handle, _stream(stream if stream is not None else self.stream)),
               "ntt_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            load().ntt_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- transforms

class Plan:
    """Transform plan of length 2^log2n mod p (owns device tables)."""

    def __init__(self, p: int, log2n: int, g: int = 0, flags: int = 0):
        L = load()
        h = ctypes.c_void_p()
        _check(L.ntt_plan_create(ctypes.byref(h), p, g, log2n, flags, None), "ntt_plan_create")
        self.handle = h
        info = PlanInfo()
        _check(L.ntt_plan_get_info(h, ctypes.byref(info)), "ntt_plan_get_info")
        self.info = info
        self.p, self.log2n, self.flags = p, log2n, flags
        self.n = 1 << log2n

    def workspace_bytes(self, batch: int = 1) -> int:
        return int(load().ntt_workspace_bytes(self.handle, batch))

    def _run(self, fn, name, x, out, batch, stride, stream, workspace):
        torch = _torch()
        if out is None:
            out = torch.empty_like(x)
        need = self.workspace_bytes(batch)
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, x.device)
        _check(fn(self.handle, _ptr(x), _ptr(out), batch, stride, _ptr(ws), ws.numel() if ws is not None else 0,
                  _stream(stream)), name)
        return out

    def forward(self, x, out=None, batch: int = 1, stride: Optional[int] = None, stream=None, workspace=None):
        return self._run(load().ntt_forward, "ntt_forward", x, out, batch, stride or self.n, stream, workspace)

    def inverse(self, x, out=None, batch: int = 1, stride: Optional[int] = None, stream=None, workspace=None):
        return self._run(load().ntt_inverse, "ntt_inverse", x, out, batch, stride or self.n, stream, workspace)

    def tft(self, x, l_out: int, l_in: Optional[int] = None, out=None, batch: int = 1, in_stride: Optional[int] = None,
            out_stride: Optional[int] = None, stream=None):
        """ntt_tft_forward: the first l_out TFT values of each of `batch` vectors of l_in
        coefficients."""
        torch = _torch()
        l_in = x.numel() // batch if l_in is None else l_in
        in_stride = in_stride or l_in or 1
        out_stride = out_stride or l_out or 1
        if out is None:
            out = torch.empty(batch * out_stride, dtype=x.dtype, device=x.device)
        L = load()
        need = int(L.ntt_tft_workspace_bytes(self.handle, batch))
        ws = _workspace(need, x.device)
        _check(L.ntt_tft_forward(self.handle, _ptr(x), l_in, _ptr(out), l_out, batch, in_stride, out_stride, _ptr(ws),
                                 need, _stream(stream)), "ntt_tft_forward")
        return out

    def itft(self, x, l: int, out=None, batch: int = 1, in_stride: Optional[int] = None,
             out_stride: Optional[int] = None, stream=None):
        """ntt_tft_inverse: the l coefficients of each vector from its first l TFT values."""
        torch = _torch()
        in_stride = in_stride or l or 1
        out_stride = out_stride or l or 1
        if out is None:
            out = torch.empty(batch * out_stride, dtype=x.dtype, device=x.device)
        L = load()
        need = int(L.ntt_tft_workspace_bytes(self.handle, batch))
        ws = _workspace(need, x.device)
        _check(L.ntt_tft_inverse(self.handle, _ptr(x), _ptr(out), l, batch, in_stride, out_stride, _ptr(ws), need,
                                 _stream(stream)), "ntt_tft_inverse")
        return out

    def close(self):
        if self.handle:
            load().ntt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
