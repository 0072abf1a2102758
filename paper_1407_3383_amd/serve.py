"""Continuous-batching server for polynomial products mod p on one GPU.

Requests (p, a, b) arrive over time with their operands in host memory.  The
scheduler admits a request when its device footprint (operands, product and
workspace) fits in the HBM budget, groups the admitted requests into one batched
launch (``polymul_modp_batch``: one fused launch per size class, several primes and
lengths together), and issues copies and launch on one of several streams.  Requests
that arrive while earlier batches run are admitted as soon as memory frees up, so
their work overlaps on the device.  Plans (twiddle tables) stay resident in the
library's cache.  Latency = arrival -> product resident in device memory.

Everything numeric runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
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
    p: int
    a: np.ndarray          # host operands (uint32 or uint64 residues)
    b: np.ndarray
    arrival: float = 0.0   # seconds since the start of the run
    admitted: float = -1.0
    done: float = -1.0
    result: Optional[object] = None  # device tensor (view into the arena) or host copy
    blocks: List = field(default_factory=list)
    bfly: int = 0


def footprint(p: int, la: int, lb: int) -> int:
    """Device bytes a request needs while in flight (operands, product, workspace)."""
    esz = 4 if p < (1 << 31) else 8
    lc = la + lb - 1
    L = ntt.load()
    ws = L.polymul_workspace_bytes(p, la, lb)
    desc = 128  # share of the batch descriptor array
    return Arena.round(la * esz) + Arena.round(lb * esz) + Arena.round(lc * esz) + Arena.round(ws) + desc


def butterflies(la: int, lb: int) -> int:
    lc = la + lb - 1
    log2n = max(0, (lc - 1).bit_length())
    return 3 * ((1 << log2n) // 2) * log2n


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
        esz = 4 if r.p < (1 << 31) else 8
        dt = torch.int32 if esz == 4 else torch.int64
        la, lb = r.a.size, r.b.size
        lc = la + lb - 1
        sizes = [la * esz, lb * esz, lc * esz]
        offs = []
        for n in sizes:
            o = self.arena.alloc(n)
            if o is None:
                for oo, nn in zip(offs, sizes):
                    self.arena.release(oo, nn)
                return False
            offs.append(o)
        r.blocks = list(zip(offs, sizes))
        r.dev = [self.arena.view(o, n, dt) for o, n in zip(offs, sizes)]
        return True

    def _release(self, r: Request):
        for o, n in r.blocks:
            self.arena.release(o, n)
        r.blocks = []

    # --------------------------------------------------------------- scheduling
    def submit(self, r: Request):
        torch = self.torch
        r.bfly = butterflies(r.a.size, r.b.size)
        view = np.int32 if r.a.dtype == np.uint32 else np.int64
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
        while self.pending and len(group) < self.max_batch:
            r = self.pending[0]
            if not self._try_admit(r):
                break
            self.pending.popleft()
            group.append(r)
            work += r.bfly
        if group:
            if not self._launch(group, now):
                return False
            return True
        return False

    def run(self, requests: List[Request], realtime: bool = True):
        """Serve `requests` (sorted by arrival); returns wall seconds of the run."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            fp = footprint(r.p, r.a.size, r.b.size)
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


def latency_stats(done: List[Request]):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    return {"p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4), "max_ms": round(float(lat.max()), 4)}
