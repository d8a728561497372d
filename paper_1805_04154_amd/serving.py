"""Serving loop: continuous batching of sort requests on one GPU.

Requests (keys + uint32 payload, key type int32 / int64 / float32) arrive
open-loop with device-resident input buffers.  The server

  * admits requests in arrival order while their bytes fit the HBM budget
    (data and scratch of every in-flight batch count against it);
  * keeps ``slots`` batches in flight at once, each on its own HIP stream with
    its own arena and workspace, so batches overlap on the device;
  * whenever a slot is free, forms a batch from the pending requests of the
    oldest request's key type (in arrival order, as many as fit the slot) and
    sorts them with one ps_segmented_sort, every request an independent
    powersort.  Requests whose buffers come from a ``RequestPool`` lie back to
    back in it in arrival order, so a batch of consecutive ones is a single
    slice of the pool and is sorted there, in place.  Other requests are
    gathered into the slot's arena and the results scattered back;
  * detects completions with events and records per-request latency from
    arrival to completion.

``serve_plain`` serves the same trace first-in first-out with one ps_sort per
request on one stream, for comparison.  Results are bit-identical either
way: a request is sorted as a segment of its own.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding

KEY_BYTES = {torch.int32: 4, torch.int64: 8, torch.float32: 4}
# HBM per admitted key: up to 8 (key) + 4 (payload) in the arena and two
# copies of both in the sort's scratch.  The sort's metadata (a few bytes
# per key at the default minimum run) is not counted.
BYTES_PER_KEY = 36


@dataclass
class ServedRequest:
    rid: int
    arrival_s: float
    keys: torch.Tensor          # device, sorted in place on completion
    payload: torch.Tensor       # device uint32, permuted alongside
    launch_s: float | None = None  # when its sort was enqueued
    done_s: float | None = None
    merge_cost: int | None = None
    pool: "RequestPool | None" = None  # the pool its buffers are slices of
    offset: int = 0                     # their first element in that pool

    @property
    def n(self) -> int:
        return int(self.keys.numel())

    @property
    def bytes(self) -> int:
        return self.n * (KEY_BYTES[self.keys.dtype] + 4)


class RequestPool:
    """Device storage for the requests of one key type: keys and a uint32
    payload, handed out back to back in the order requests are made.  The
    caller fills a request's buffers before submitting it; the server sorts
    runs of consecutive requests in place as one segmented sort."""

    def __init__(self, dtype: torch.dtype, capacity: int, device="cuda"):
        if dtype not in KEY_BYTES:
            raise ValueError(f"unsupported key type {dtype}")
        self.dtype = dtype
        self.capacity = int(capacity)
        self.keys = torch.empty(self.capacity, dtype=dtype, device=device)
        self.payload = torch.empty(self.capacity, dtype=torch.int32, device=device).view(torch.uint32)
        self.used = 0

    def request(self, rid: int, arrival_s: float, n: int) -> ServedRequest:
        """A request of n keys whose buffers are the pool's next n elements."""
        if self.used + n > self.capacity:
            raise ValueError(f"pool of {self.capacity} keys has {self.capacity - self.used} left, asked for {n}")
        a = self.used
        self.used += n
        return ServedRequest(rid, arrival_s, self.keys[a:a + n], self.payload[a:a + n], pool=self, offset=a)

    def reset(self):
        """Start handing out from the front again (earlier requests' buffers
        are reused, so they must be finished with)."""
        self.used = 0


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    arena_keys: torch.Tensor    # raw bytes for keys
    arena_pay: torch.Tensor     # uint32
    workspace: torch.Tensor
    capacity: int               # keys per batch (key bytes <= 8)
    batch: list = field(default_factory=list)
    event: torch.cuda.Event | None = None
    costs: torch.Tensor | None = None
    budget_held: int = 0
    start_s: float = 0.0
    off_host: torch.Tensor | None = None  # pinned offsets, alive until the batch completes


class SortServer:
    """Continuous-batching sort server (one GPU, several in-flight batches)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 2, max_batch_keys: int | None = None,
                 min_run: int | None = None, max_segments: int = 4096, device="cuda"):
        binding.load_library()
        self.budget = int(hbm_budget_bytes)
        self.min_run = min_run
        self.max_segments = max_segments
        per_slot = self.budget // max(slots, 1)
        cap = per_slot // BYTES_PER_KEY
        if max_batch_keys:
            cap = min(cap, int(max_batch_keys))
        if cap < 1:
            raise ValueError("HBM budget too small")
        self.slots: list[_Slot] = []
        for _ in range(slots):
            ws = binding.workspace_bytes(cap, max_segments, torch.int64, True, min_run)
            self.slots.append(_Slot(stream=torch.cuda.Stream(device=device),
                                    arena_keys=torch.empty(cap * 8, dtype=torch.uint8, device=device),
                                    arena_pay=torch.empty(cap, dtype=torch.int32, device=device).view(torch.uint32),
                                    workspace=torch.empty(ws, dtype=torch.uint8, device=device),
                                    capacity=cap))
        self.in_use = 0
        self.busy_s = 0.0

    # ------------------------------------------------------------------ batches

    @staticmethod
    def _in_place(batch: list[ServedRequest]) -> bool:
        """True if the batch is consecutive requests of one pool."""
        pool = batch[0].pool
        if pool is None:
            return False
        end = batch[0].offset
        for r in batch:
            if r.pool is not pool or r.offset != end:
                return False
            end += r.n
        return True

    def _launch(self, slot: _Slot, batch: list[ServedRequest], now: float):
        dt = batch[0].keys.dtype
        kb = KEY_BYTES[dt]
        sizes = [r.n for r in batch]
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum(sizes)
        total = int(offs[-1])
        in_place = self._in_place(batch)
        if in_place:
            a0 = batch[0].offset
            keys, pay = batch[0].pool.keys[a0:a0 + total], batch[0].pool.payload[a0:a0 + total]
        else:
            keys = slot.arena_keys[: total * kb].view(dt)
            pay = slot.arena_pay[:total]
        main = torch.cuda.current_stream()
        slot.stream.wait_stream(main)  # request buffers were produced on the caller's stream
        with torch.cuda.stream(slot.stream):
            if not in_place:
                for r, a, b in zip(batch, offs[:-1], offs[1:]):
                    keys[a:b].copy_(r.keys)
                    pay[a:b].copy_(r.payload)
            # pinned + non-blocking: the host does not wait for queued work
            off_h = torch.from_numpy(offs).pin_memory()
            off_t = off_h.to(keys.device, non_blocking=True)
            slot.off_host = off_h
            costs = torch.zeros(len(batch), dtype=torch.int64, device=keys.device)
            binding.segmented_sort(keys, pay, off_t, min_run=self.min_run, merge_costs=costs,
                                   stream=slot.stream, workspace=slot.workspace)
            if not in_place:
                for r, a, b in zip(batch, offs[:-1], offs[1:]):
                    r.keys.copy_(keys[a:b])
                    r.payload.copy_(pay[a:b])
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.batch, slot.event, slot.costs, slot.start_s = batch, ev, costs, now
        for r in batch:
            r.launch_s = now

    def _poll(self, slot: _Slot, now: float, done: list):
        if slot.event is None or not slot.event.query():
            return False
        costs = slot.costs.cpu().numpy().view(np.uint64)
        for r, c in zip(slot.batch, costs):
            r.done_s = now
            r.merge_cost = int(c)
            done.append(r)
        self.busy_s += now - slot.start_s
        self.in_use -= slot.budget_held
        slot.batch, slot.event, slot.costs, slot.budget_held, slot.off_host = [], None, None, 0, None
        return True

    # --------------------------------------------------------------------- loop

    def serve(self, requests: list[ServedRequest], realtime: bool = True) -> list[ServedRequest]:
        """Serve an open-loop trace (requests sorted by arrival).  Returns the
        completed requests in completion order; latencies are done_s - arrival_s.
        With realtime=False every request is available at time 0 (saturation)
        and its arrival_s is set to 0."""
        if not realtime:
            for r in requests:
                r.arrival_s = 0.0
        torch.cuda.synchronize()
        pending: list[ServedRequest] = []
        done: list[ServedRequest] = []
        nxt = 0
        t0 = time.perf_counter()
        total = len(requests)
        while len(done) < total:
            now = time.perf_counter() - t0
            while nxt < total and (requests[nxt].arrival_s <= now or not realtime):
                pending.append(requests[nxt])
                nxt += 1
            progressed = False
            for s in self.slots:
                progressed |= self._poll(s, now, done)
            for s in self.slots:
                if s.event is not None or not pending:
                    continue
                dt = pending[0].keys.dtype
                batch, keys, held = [], 0, 0
                rest = []
                for r in pending:
                    fits_slot = r.keys.dtype == dt and keys + r.n <= s.capacity and len(batch) < self.max_segments
                    if fits_slot and batch and batch[0].pool is not None:
                        # a pool batch stays one slice: only the next request of that pool joins it
                        last = batch[-1]
                        fits_slot = r.pool is last.pool and r.offset == last.offset + last.n
                    need = BYTES_PER_KEY * r.n  # as in the slot sizing
                    if fits_slot and self.in_use + held + need <= self.budget:
                        batch.append(r)
                        keys += r.n
                        held += need
                    else:
                        rest.append(r)
                if not batch:
                    head = pending[0]
                    if head.n > s.capacity:
                        raise ValueError(f"request of {head.n} keys exceeds a batch slot ({s.capacity})")
                    if all(x.event is None for x in self.slots) and self.in_use == 0:
                        raise RuntimeError("nothing in flight and the oldest request does not fit the budget")
                    continue
                pending = rest
                self.in_use += held
                s.budget_held = held
                self._launch(s, batch, now)
                progressed = True
            if not progressed:
                time.sleep(2e-5)
        return done


def serve_plain(requests: list[ServedRequest], min_run: int | None = None, realtime: bool = True):
    """FIFO, one ps_sort per request on the current stream, no batching.
    realtime=False: every request is available at time 0 (arrival_s set to 0)."""
    if not realtime:
        for r in requests:
            r.arrival_s = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = []
    inflight = []
    nxt = 0
    s = torch.cuda.current_stream()
    while len(done) < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(requests) and (requests[nxt].arrival_s <= now or not realtime):
            r = requests[nxt]
            M = torch.zeros(1, dtype=torch.int64, device=r.keys.device)
            r.launch_s = now
            binding.sort(r.keys, r.payload, min_run=min_run, merge_cost=M)
            ev = torch.cuda.Event()
            ev.record(s)
            inflight.append((r, ev, M))
            nxt += 1
        now = time.perf_counter() - t0
        keep = []
        for r, ev, M in inflight:
            if ev.query():
                r.done_s = now
                r.merge_cost = int(M.item())
                done.append(r)
            else:
                keep.append((r, ev, M))
        inflight = keep
        if nxt < len(requests) and not inflight:
            time.sleep(2e-5)
    return done


def busy_time(intervals: list[tuple[float, float]]) -> float:
    """Length of the union of [start, end) intervals, e.g. (launch_s, done_s)
    of served requests: the host-observed time with work in flight."""
    total, cur_s, cur_e = 0.0, None, None
    for s, e in sorted(intervals):
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                total += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        total += cur_e - cur_s
    return total


def algorithmic_bytes(done: list[ServedRequest]) -> int:
    """Sum over requests of (K+V)(2M + 2n): each merge reads its inputs and
    writes its result, plus one pass for run detection and leaf formation."""
    return sum((KEY_BYTES[r.keys.dtype] + 4) * (2 * int(r.merge_cost) + 2 * r.n) for r in done)


def latency_stats(done: list[ServedRequest], hbm_peak_bps: float = 8.0e12) -> dict:
    """p50/p99/mean latency (arrival to completion), keys/s over the span, and
    the roofline fraction of the algorithmic bytes over the busy time."""
    lat = np.array([r.done_s - r.arrival_s for r in done]) * 1e3
    keys = sum(r.n for r in done)
    span = max(r.done_s for r in done) - min(r.arrival_s for r in done)
    busy = busy_time([(r.launch_s, r.done_s) for r in done])
    b_alg = algorithmic_bytes(done)
    return {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "keys": int(keys), "span_s": round(span, 4), "keys_per_s": round(keys / span, 1),
            "busy_s": round(busy, 4), "algorithmic_bytes": int(b_alg),
            "busy_roofline_frac": round(b_alg / busy / hbm_peak_bps, 4) if busy > 0 else None}
