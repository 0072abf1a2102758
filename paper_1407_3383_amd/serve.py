"""Continuous-batching server for polynomial and integer products on one GPU.

Requests arrive over time with their operands in host memory: polynomial products
(p, a, b) and integer products (16-bit limbs a, b; ``Request.kind == "int"``).  The
scheduler admits a request when its device footprint (operands, product and
workspace) fits in the HBM budget, groups the admitted polynomial requests into one
batched launch (``polymul_modp_batch``: one fused launch per size class, several
primes and lengths together), issues each admitted integer product as one
``intmul_crt`` call, and spreads copies and launches over several streams.  Requests
that arrive while earlier work runs are admitted as soon as memory frees up, so
their work overlaps on the device.  Plans (twiddle tables) stay resident in the
library's cache.  Latency = arrival -> product resident in device memory.

Everything numeric runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import ntt

ALIGN = 256


class Arena:
    """First-fit allocator over one device buffer of `budget` bytes (the HBM budget)."""

    def __init__(self, budget: int, device="cuda"):
        import torch
        self.budget = budget
        self.buf = torch.empty(budget, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.free = [(0, budget)]  # sorted (offset, size)
        self.used = 0

    @staticmethod
    def round(n: int) -> int:
        return (max(n, 1) + ALIGN - 1) // ALIGN * ALIGN

    def alloc(self, n: int) -> Optional[int]:
        n = self.round(n)
        for i, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, size - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int):
        n = self.round(n)
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def view(self, off: int, nbytes: int, dtype):
        import torch
        return self.buf[off:off + nbytes].view(dtype)


@dataclass
class Request:
    rid: int
    p: int                 # prime of a polynomial product (ignored for "int")
    a: np.ndarray          # host operands: uint32/uint64 residues, or uint16 limbs
    b: np.ndarray
    arrival: float = 0.0   # seconds since the start of the run
    admitted: float = -1.0
    done: float = -1.0
    result: Optional[object] = None  # device tensor (view into the arena) or host copy
    blocks: List = field(default_factory=list)
    bfly: int = 0
    kind: str = "poly"     # "poly" (product mod p) or "int" (integer product)


def footprint(p: int, la: int, lb: int) -> int:
    """Device bytes a request needs while in flight (operands, product, workspace)."""
    esz = 4 if p < (1 << 31) else 8
    lc = la + lb - 1
    L = ntt.load()
    ws = L.polymul_workspace_bytes(p, la, lb)
    desc = 128  # share of the batch descriptor array
    return Arena.round(la * esz) + Arena.round(lb * esz) + Arena.round(lc * esz) + Arena.round(ws) + desc


def int_footprint(na: int, nb: int) -> int:
    """Device bytes of an integer product in flight (limbs, product limbs, workspace)."""
    L = ntt.load()
    nc = (na + nb + 1) // 2
    return (Arena.round(2 * na) + Arena.round(2 * nb) + Arena.round(4 * nc)
            + Arena.round(L.intmul_workspace_bytes(na, nb)))


def request_footprint(r: "Request") -> int:
    if r.kind == "int":
        return int_footprint(r.a.size, r.b.size)
    return footprint(r.p, r.a.size, r.b.size)


def butterflies(la: int, lb: int, primes: int = 1) -> int:
    lc = la + lb - 1
    log2n = max(0, (lc - 1).bit_length())
    return primes * 3 * ((1 << log2n) // 2) * log2n


class Server:
    def __init__(self, budget_bytes: int, streams: int = 4, max_batch: int = 256, keep_results: bool = True):
        import torch
        self.torch = torch
        self.arena = Arena(budget_bytes)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]  # default priority
        self.next_stream = 0
        self.max_batch = max_batch
        self.keep_results = keep_results
        self.pending = collections.deque()
        self.inflight = []  # (event, [requests], ws_block)
        self.completed: List[Request] = []
        self.max_inflight_batches = 0
        self.overlapped_admissions = 0

    # --------------------------------------------------------------- memory
    def _try_admit(self, r: Request) -> bool:
        torch = self.torch
        la, lb = r.a.size, r.b.size
        if r.kind == "int":
            nc = (la + lb + 1) // 2
            ws = ntt.load().intmul_workspace_bytes(la, lb)
            sizes = [2 * la, 2 * lb, 4 * nc, max(ws, 1)]
            dts = [torch.int16, torch.int16, torch.int32, torch.uint8]
        else:
            esz = 4 if r.p < (1 << 31) else 8
            dt = torch.int32 if esz == 4 else torch.int64
            lc = la + lb - 1
            sizes = [la * esz, lb * esz, lc * esz]
            dts = [dt, dt, dt]
        offs = []
        for n in sizes:
            o = self.arena.alloc(n)
            if o is None:
                for oo, nn in zip(offs, sizes):
                    self.arena.release(oo, nn)
                return False
            offs.append(o)
        r.blocks = list(zip(offs, sizes))
        r.dev = [self.arena.view(o, n, t) for o, n, t in zip(offs, sizes, dts)]
        return True

    def _release(self, r: Request):
        for o, n in r.blocks:
            self.arena.release(o, n)
        r.blocks = []

    # --------------------------------------------------------------- scheduling
    def submit(self, r: Request):
        torch = self.torch
        r.bfly = butterflies(r.a.size, r.b.size, 3 if r.kind == "int" else 1)
        view = {np.dtype(np.uint16): np.int16, np.dtype(np.uint32): np.int32,
                np.dtype(np.uint64): np.int64}[np.dtype(r.a.dtype)]
        # page-locked host copies so the uploads are true asynchronous DMA
        r.ha = torch.from_numpy(np.ascontiguousarray(r.a).view(view)).pin_memory()
        r.hb = torch.from_numpy(np.ascontiguousarray(r.b).view(view)).pin_memory()
        self.pending.append(r)

    def _launch(self, group: List[Request], now: float):
        torch = self.torch
        L = ntt.load()

        def descs_of(g):
            d = (ntt.PolymulDesc * len(g))()
            for i, r in enumerate(g):
                a, b, c = r.dev
                d[i] = ntt.PolymulDesc(r.p, a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), c.data_ptr())
            return d

        # the batch scratch; shrink the group until it fits next to what is in flight
        descs = descs_of(group)
        need = L.polymul_batch_workspace_bytes(descs, len(group))
        ws_off = self.arena.alloc(need) if need else None
        while need and ws_off is None and len(group) > 1:
            r = group.pop()
            self._release(r)
            self.pending.appendleft(r)
            descs = descs_of(group)
            need = L.polymul_batch_workspace_bytes(descs, len(group))
            ws_off = self.arena.alloc(need) if need else None
        if need and ws_off is None:
            for r in reversed(group):
                self._release(r)
                self.pending.appendleft(r)
            return False
        s = self.streams[self.next_stream % len(self.streams)]
        self.next_stream += 1
        with torch.cuda.stream(s):
            for r in group:
                r.dev[0].copy_(r.ha, non_blocking=True)
                r.dev[1].copy_(r.hb, non_blocking=True)
        ws_ptr = (self.arena.base + ws_off) if need else None
        ntt._check(L.polymul_modp_batch(descs, len(group), ws_ptr, need, ntt._stream(s)), "polymul_modp_batch")
        ev = torch.cuda.Event()
        ev.record(s)
        if self.inflight:
            self.overlapped_admissions += len(group)
        self.inflight.append((ev, group, (ws_off, need) if need else None, s))
        self.max_inflight_batches = max(self.max_inflight_batches, len(self.inflight))
        for r in group:
            r.admitted = now
        return True

    def _launch_int(self, r: Request, now: float):
        torch = self.torch
        L = ntt.load()
        s = self.streams[self.next_stream % len(self.streams)]
        self.next_stream += 1
        a, b, c, ws = r.dev
        with torch.cuda.stream(s):
            a.copy_(r.ha, non_blocking=True)
            b.copy_(r.hb, non_blocking=True)
        ntt._check(L.intmul_crt(ntt._ptr(a), a.numel(), ntt._ptr(b), b.numel(), ntt._ptr(c), ntt._ptr(ws),
                                ws.numel(), ntt._stream(s)), "intmul_crt")
        ev = torch.cuda.Event()
        ev.record(s)
        if self.inflight:
            self.overlapped_admissions += 1
        self.inflight.append((ev, [r], None, s))
        self.max_inflight_batches = max(self.max_inflight_batches, len(self.inflight))
        r.admitted = now

    def _poll(self, now_fn):
        still = []
        for ev, group, ws, s in self.inflight:
            if ev.query():
                t = now_fn()
                for r in group:
                    r.done = t
                    if self.keep_results:
                        # synchronous copy to the host before the arena block is reused
                        r.result = ntt.to_numpy(r.dev[2])
                        if r.kind == "int":
                            r.result = r.result.astype(np.uint32)
                    self._release(r)
                    r.dev = None
                    r.ha = r.hb = None
                    self.completed.append(r)
                if ws:
                    self.arena.release(*ws)
            else:
                still.append((ev, group, ws, s))
        self.inflight = still

    def _admit_and_launch(self, now: float):
        group, work = [], 0
        launched = False
        while self.pending and len(group) < self.max_batch:
            r = self.pending[0]
            if not self._try_admit(r):
                break
            self.pending.popleft()
            if r.kind == "int":
                self._launch_int(r, now)
                launched = True
                continue
            group.append(r)
            work += r.bfly
        if group:
            return self._launch(group, now) or launched
        return launched

    def run(self, requests: List[Request], realtime: bool = True):
        """Serve `requests` (sorted by arrival); returns wall seconds of the run."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            fp = request_footprint(r)
            if fp > self.arena.budget:
                raise ValueError("request %d needs %d bytes, more than the HBM budget %d" % (r.rid, fp, self.arena.budget))
        t0 = time.perf_counter()
        now_fn = lambda: time.perf_counter() - t0
        i = 0
        total = len(reqs)
        while len(self.completed) < total:
            now = now_fn()
            while i < total and (not realtime or reqs[i].arrival <= now):
                self.submit(reqs[i])
                i += 1
            self._poll(now_fn)
            launched = self._admit_and_launch(now_fn())
            if not launched and not self.inflight and not self.pending and i < total and realtime:
                time.sleep(max(0.0, min(reqs[i].arrival - now_fn(), 0.001)))
        self.torch.cuda.synchronize()
        return now_fn()


class NativeServer:
    """The same request loop in the library (ntt_server_*): admission, batching, staging
    and completion run in native code; this class only feeds arrivals and collects
    completions.  Results always come back to host arrays (Request.result)."""

    def __init__(self, budget_bytes: int, streams: int = 4, max_batch: int = 64, keep_results: bool = True,
                 pinned_results: bool = False):
        """pinned_results: result arrays in page-locked memory, which the server fills by
        DMA directly (no staging copy)."""
        import torch
        self.torch = torch
        self.pinned_results = pinned_results
        L = ntt.load()
        h = ctypes.c_void_p()
        ntt._check(L.ntt_server_create(ctypes.byref(h), budget_bytes, streams, max_batch), "ntt_server_create")
        self.h = h
        self.budget = budget_bytes
        self.keep_results = keep_results
        self.completed: List[Request] = []
        self.max_inflight_batches = 0

    def stats(self):
        L = ntt.load()
        v = [ctypes.c_size_t() for _ in range(4)]
        ntt._check(L.ntt_server_stats(self.h, *[ctypes.byref(x) for x in v]), "ntt_server_stats")
        return {"pending": v[0].value, "inflight": v[1].value, "arena_used": v[2].value,
                "max_inflight": v[3].value}

    def run(self, requests: List[Request], realtime: bool = True):
        """Serve `requests` (sorted by arrival); returns wall seconds of the run."""
        L = ntt.load()
        reqs = sorted(requests, key=lambda r: r.arrival)
        byid = {}
        for r in reqs:
            n = (r.a.size + r.b.size + 1) // 2 if r.kind == "int" else r.a.size + r.b.size - 1
            dt = np.uint32 if (r.kind == "int" or r.p < (1 << 31)) else np.uint64
            # result buffers touched before the run, so that no page is first touched
            # by the copy-back inside it
            # (a result array the request already carries, of the right size and type,
            # is reused: callers that serve the same requests again keep their buffers)
            reuse = (self.keep_results and not self.pinned_results and isinstance(r.result, np.ndarray)
                     and r.result.size == n and r.result.dtype == dt)
            if not reuse:
                r.result = None
            if self.keep_results and self.pinned_results:
                tdt = self.torch.int32 if dt == np.uint32 else self.torch.int64
                r._pinned = self.torch.empty(n, dtype=tdt, pin_memory=True)
                r.result = r._pinned.numpy().view(dt)
            elif self.keep_results and not reuse:
                r.result = np.zeros(n, dtype=dt)
                r.result.fill(1)
            r.a = np.ascontiguousarray(r.a)
            r.b = np.ascontiguousarray(r.b)
            r.bfly = butterflies(r.a.size, r.b.size, 3 if r.kind == "int" else 1)
            byid[r.rid] = r
        cap = 4096
        ids = (ctypes.c_uint64 * cap)()
        nd = ctypes.c_size_t()
        t0 = time.perf_counter()
        i, total, done = 0, len(reqs), 0
        while done < total:
            now = time.perf_counter() - t0
            while i < total and (not realtime or reqs[i].arrival <= now):
                r = reqs[i]
                rc = L.ntt_server_submit(self.h, r.rid, 1 if r.kind == "int" else 0, r.p,
                                         r.a.ctypes.data, r.a.size, r.b.ctypes.data, r.b.size,
                                         r.result.ctypes.data if r.result is not None else None)
                if rc != ntt.NTT_OK:
                    raise ValueError("request %d refused by the server (%d)" % (r.rid, rc))
                r.admitted = now
                i += 1
            ntt._check(L.ntt_server_progress(self.h, ids, cap, ctypes.byref(nd)), "ntt_server_progress")
            if nd.value:
                t = time.perf_counter() - t0
                for k in range(nd.value):
                    r = byid[ids[k]]
                    r.done = t
                    self.completed.append(r)
                done += nd.value
            elif i < total and realtime and done == i:
                time.sleep(max(0.0, min(reqs[i].arrival - (time.perf_counter() - t0), 0.0005)))
        self.max_inflight_batches = self.stats()["max_inflight"]
        return time.perf_counter() - t0

    def close(self):
        if getattr(self, "h", None):
            ntt.load().ntt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latency_stats(done: List[Request]):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    return {"p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4), "max_ms": round(float(lat.max()), 4)}
