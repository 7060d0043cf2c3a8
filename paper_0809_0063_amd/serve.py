"""Continuous-batching request loop over the packed F_p kernels.

Requests reference payloads (an F_p matrix product or a batch of polynomial
products) and arrive on a Poisson clock.  The loop

* admits an arrived request when a slot is free and its device memory fits the
  HBM budget (operands, output, packed workspace); a request that does not fit
  waits, it is never dropped;
* keeps packed operands resident: the packed words of a product's B operand
  (and the device copies of every operand) stay in a residency cache keyed by
  payload, evicted least-recently-used when the budget needs room, so a
  repeated payload skips its upload and packing;
* cuts every matrix product into row chunks of bounded work (at most
  `chunk_macs` multiply-adds per launch), so a large product never holds the
  device for long and small requests are interleaved with it;
* launches each step's chunks on the streams of their slots (one stream per
  slot, several slots in flight), so the work of different requests overlaps
  on the device, and detects completion with events;
* records arrival-to-completion latency per request (p50/p99) and throughput.

The result bytes of a request do not depend on what else runs: every chunk
writes only its own rows of its own output.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import dqt as D
from . import inputs


@dataclass
class Request:
    rid: int
    item: int                 # pool index
    arrival: float            # seconds from the start of the run
    admitted: float = -1.0
    done: float = -1.0
    slot: int = -1
    chunks: List = field(default_factory=list)
    next_chunk: int = 0
    event: Optional[torch.cuda.Event] = None
    out: Optional[torch.Tensor] = None
    bytes: int = 0
    # device buffers held while the request is active (released at completion;
    # the residency cache keeps its own references to cached operands)
    A: Optional[torch.Tensor] = None
    B: Optional[torch.Tensor] = None
    CA: Optional[torch.Tensor] = None
    CB: Optional[torch.Tensor] = None
    stream: Optional[torch.cuda.Stream] = None


class ResidencyCache:
    """Device copies of payload operands and packed B words, LRU under a byte budget."""

    def __init__(self, budget: int):
        self.budget = budget
        self.used = 0
        self.entries: "collections.OrderedDict[tuple, tuple]" = collections.OrderedDict()
        self.hits = 0
        self.misses = 0

    def get(self, key):
        ent = self.entries.get(key)
        if ent is not None:
            self.entries.move_to_end(key)
            self.hits += 1
            return ent[0]
        self.misses += 1
        return None

    def put(self, key, value, nbytes: int, pinned: set):
        while self.used + nbytes > self.budget and self._evict_one(pinned):
            pass
        if self.used + nbytes > self.budget:
            return False
        self.entries[key] = (value, nbytes)
        self.used += nbytes
        return True

    def _evict_one(self, pinned: set) -> bool:
        for k in list(self.entries.keys()):
            if k[0] in pinned:
                continue
            _, nb = self.entries.pop(k)
            self.used -= nb
            return True
        return False


class Server:
    def __init__(self, pool: Sequence[inputs.Payload], hbm_budget: int = 16 << 30, slots: int = 8,
                 chunk_macs: int = 1 << 28, cache_fraction: float = 0.5, pregenerate: bool = True):
        self.pool = list(pool)
        # The clients' payloads live in pinned host memory before the run starts (a request
        # whose operands are not resident pays only their upload, not their generation).
        self.host_ops = None
        if pregenerate:
            self.host_ops = []
            for pl in self.pool:
                a, b = inputs.payload_operands(pl)
                self.host_ops.append((torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory()))
        self.dev = torch.device("cuda:0")
        self.hbm_budget = int(hbm_budget)
        self.cache = ResidencyCache(int(hbm_budget * cache_fraction))
        self.active_budget = self.hbm_budget - self.cache.budget
        self.active_bytes = 0
        self.slots = slots
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.chunk_macs = chunk_macs
        self.plan = D.GemmPlan()  # AUTO: packed when the bounds allow it

    # --- operands ------------------------------------------------------------

    def _operands(self, i: int, pinned: set, stream):
        key = (i, "ops")
        ent = self.cache.get(key)
        if ent is None:
            if self.host_ops is not None:
                ha, hb = self.host_ops[i]
            else:
                a, b = inputs.payload_operands(self.pool[i])
                ha, hb = torch.from_numpy(a), torch.from_numpy(b)
            # uploaded on the request's stream; later users on other streams wait for it
            with torch.cuda.stream(stream):
                A = ha.to(self.dev, non_blocking=True)
                B = hb.to(self.dev, non_blocking=True)
                ready = torch.cuda.Event()
                ready.record(stream)
            self.cache.put(key, (A, B, ready), A.numel() + B.numel(), pinned)
            return A, B
        A, B, ready = ent
        stream.wait_event(ready)
        A.record_stream(stream)
        B.record_stream(stream)
        return A, B

    def _packed_b(self, i: int, B: torch.Tensor, p: int, stream, pinned: set) -> torch.Tensor:
        key = (i, "CB")
        ent = self.cache.get(key)
        if ent is None:
            with torch.cuda.stream(stream):
                CB = D.fgemm_pack_side(B, p, 1, plan=self.plan)
                ready = torch.cuda.Event()
                ready.record(stream)
            self.cache.put(key, (CB, ready), CB.numel(), pinned)
            return CB
        CB, ready = ent
        # packed on another slot's stream: order this stream after the packing, and
        # keep the allocator from reusing the buffer before this stream is done with it
        stream.wait_event(ready)
        CB.record_stream(stream)
        return CB

    def _gemm_chunk_rows(self, n: int) -> int:
        rows = max(16, int(self.chunk_macs // max(1, n * n)))
        rows = (rows // 16) * 16
        return max(16, min(n, rows))

    def _request_bytes(self, pl: inputs.Payload) -> int:
        if pl.kind == "gemm":
            n = pl.n
            rows = self._gemm_chunk_rows(n)
            ca = D.fgemm_packed_bytes(pl.p, rows, n, 0, self.plan)
            return n * n + ca + 2 * n * n
        return pl.n * (2 * pl.deg + 1) + 2 * pl.n * (pl.deg + 1)

    # --- request set-up ---------------------------------------------------------

    def _prepare(self, r: Request, pinned: set):
        pl = self.pool[r.item]
        s = self.streams[r.slot]
        A, B = self._operands(r.item, pinned, s)
        if pl.kind == "gemm":
            n = pl.n
            r.out = torch.empty((n, n), dtype=torch.uint8, device=self.dev)
            rows = self._gemm_chunk_rows(n)
            r.chunks = [(r0, min(n, r0 + rows)) for r0 in range(0, n, rows)]
            r.CB = self._packed_b(r.item, B, pl.p, s, pinned)
            r.CA = torch.empty(D.fgemm_packed_bytes(pl.p, rows, n, 0, self.plan), dtype=torch.uint8,
                               device=self.dev)
        else:
            r.out = torch.empty((pl.n, 2 * pl.deg + 1), dtype=torch.uint8, device=self.dev)
            r.chunks = [None]
        r.A, r.B = A, B
        r.stream = s

    def _launch_chunk(self, r: Request):
        pl = self.pool[r.item]
        c = r.chunks[r.next_chunk]
        with torch.cuda.stream(r.stream):
            if pl.kind == "gemm":
                r0, r1 = c
                m = r1 - r0
                # the rows of this chunk are packed into the request's buffer (the stream orders the
                # reuse of that buffer by the next chunk); B stays packed in the residency cache
                D.fgemm_pack_side(r.A[r0:r1], pl.p, 0, plan=self.plan, out=r.CA)
                D.fgemm_packed(r.CA, r.CB, pl.p, m, pl.n, pl.n, plan=self.plan, out=r.out[r0:r1])
            else:
                polymul(r.A, r.B, pl.p, out=r.out)
        r.next_chunk += 1
        if r.next_chunk == len(r.chunks):
            r.event = torch.cuda.Event()
            r.event.record(r.stream)

    # --- the loop -----------------------------------------------------------------

    def run(self, arrivals: np.ndarray, items: np.ndarray, max_wall: float = 600.0, warmup: int = 0,
            on_step=None):
        """Serve the requests; `on_step(active, finished)`, if given, is called once per loop pass."""
        reqs = [Request(i, int(it), float(t)) for i, (t, it) in enumerate(zip(arrivals, items))]
        pending = collections.deque(reqs)
        waiting: collections.deque = collections.deque()
        active: List[Request] = []
        finished: List[Request] = []
        t0 = time.perf_counter()
        while (pending or waiting or active) and time.perf_counter() - t0 < max_wall:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: a free slot and room in the HBM budget
            while waiting and self.free_slots:
                r = waiting[0]
                need = self._request_bytes(self.pool[r.item])
                if self.active_bytes + need > self.active_budget and active:
                    break
                waiting.popleft()
                r.slot = self.free_slots.pop()
                r.bytes = need
                r.admitted = now
                self.active_bytes += need
                self._prepare(r, {a.item for a in active} | {r.item})
                active.append(r)
            # one step: the next chunk of every active request that has one
            for r in active:
                if r.next_chunk < len(r.chunks):
                    self._launch_chunk(r)
            # completions
            still = []
            for r in active:
                if r.event is not None and r.event.query():
                    r.done = time.perf_counter() - t0
                    self.free_slots.append(r.slot)
                    self.active_bytes -= r.bytes
                    # only the output outlives the request: its operands and packed words go
                    # back to the allocator (or stay only as far as the cache holds them)
                    r.A = r.B = r.CA = r.CB = None
                    r.stream = None
                    finished.append(r)
                else:
                    still.append(r)
            active = still
            if on_step is not None:
                on_step(active, finished)
            if not active and waiting == collections.deque() and pending:
                # idle until the next arrival
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
        torch.cuda.synchronize()
        self.wall = time.perf_counter() - t0
        return finished

    @staticmethod
    def summary(finished: List[Request], warmup: int, pool) -> Dict[str, float]:
        measured = [r for r in finished if r.rid >= warmup]
        lat = np.array([r.done - r.arrival for r in measured]) if measured else np.zeros(1)
        span = (max(r.done for r in measured) - min(r.arrival for r in measured)) if measured else 1.0
        ops = 0.0
        for r in measured:
            pl = pool[r.item]
            ops += 2.0 * pl.n ** 3 if pl.kind == "gemm" else 2.0 * pl.n * (pl.deg + 1) ** 2
        return {"requests": len(measured), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "req_per_s": len(measured) / span if span > 0 else 0.0, "fp_gop_s": ops / span / 1e9 if span > 0 else 0.0}


def polymul(a: torch.Tensor, b: torch.Tensor, p: int, out: torch.Tensor):
    """Polynomial products of any degree up to 63: one word when it fits, FQT blocks otherwise, plain last."""
    k = a.shape[1]
    try:
        return D.polymul_u8(a, b, p, out=out)
    except D.DQTError as e:
        if e.status != D.DQT_E_UNSUPPORTED:
            raise
    try:
        return D.polymul_fqt_u8(a, b, p, out=out)
    except D.DQTError as e:
        if e.status != D.DQT_E_UNSUPPORTED:
            raise
    return D.polymul_plain_u8(a, b, p, out=out)


def run_alone(server: Server, item: int) -> torch.Tensor:
    """One payload on its own (fresh output, null stream), for the alone-vs-mix comparison."""
    pl = server.pool[item]
    if server.host_ops is not None:
        ha, hb = server.host_ops[item]
    else:
        a, b = inputs.payload_operands(pl)
        ha, hb = torch.from_numpy(a), torch.from_numpy(b)
    A, B = ha.to(server.dev), hb.to(server.dev)
    if pl.kind == "gemm":
        return D.fgemm(A, B, pl.p)
    out = torch.empty((pl.n, 2 * pl.deg + 1), dtype=torch.uint8, device=server.dev)
    return polymul(A, B, pl.p, out)
