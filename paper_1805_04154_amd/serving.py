"""Serving loop: continuous batching of sort requests on one GPU.

Requests (keys + uint32 payload, key type int32 / int64 / float32) arrive
open-loop with device-resident input buffers.  The server

  * owns one device arena of exactly its HBM budget and carves every batch's
    memory out of it: the sort's workspace (``ps_workspace_bytes`` for the
    batch's own key type, size and segment count) and, for requests that
    must be gathered, their keys and payloads.  A batch is admitted only
    while its bytes fit a free block of the arena, so in-flight memory never
    exceeds the budget, and a free slot waits when memory, not slots, runs
    out;
  * keeps ``slots`` batches in flight at once, each on its own HIP stream, so
    batches overlap on the device;
  * whenever a slot is free, forms a batch from the pending requests of the
    oldest request's key type (in arrival order, as many as fit the free
    memory) and sorts them with one ps_segmented_sort, every request an
    independent powersort.  Requests whose buffers come from a
    ``RequestPool`` lie back to back in it in arrival order, so a batch of
    consecutive ones is a single slice of the pool and is sorted there, in
    place.  Other requests are gathered into arena memory and the results
    scattered back;
  * detects completions with events and records per-request latency from
    arrival to completion, and each batch's interval on the device (timing
    events on its stream before its first and after its last launch).

``serve_plain`` serves the same trace first-in first-out with one ps_sort per
request on one stream, for comparison.  Results are bit-identical either
way: a request is sorted as a segment of its own.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding

KEY_BYTES = {torch.int32: 4, torch.int64: 8, torch.float32: 4}
ALIGN = 256  # arena blocks and the parts inside them start on 256-byte boundaries


def _align(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


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


class ArenaAllocator:
    """First-fit placement of blocks in [0, size) (host-side bookkeeping of
    the server's device arena).  Free blocks are kept sorted by offset and
    coalesced with their neighbours on release."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free: list[tuple[int, int]] = [(0, self.size)] if self.size > 0 else []
        self.in_use = 0

    def largest_free(self) -> int:
        return max((n for _, n in self.free), default=0)

    def alloc(self, nbytes: int) -> int | None:
        """Offset of a new block of nbytes (rounded up to ALIGN), or None."""
        need = _align(max(nbytes, 1))
        for i, (off, n) in enumerate(self.free):
            if n >= need:
                if n == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, n - need)
                self.in_use += need
                return off
        return None

    def release(self, off: int, nbytes: int):
        need = _align(max(nbytes, 1))
        i = bisect.bisect_left(self.free, (off, 0))
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] > off:
            raise ValueError("block overlaps a free block")
        if i < len(self.free) and off + need > self.free[i][0]:
            raise ValueError("block overlaps a free block")
        self.free.insert(i, (off, need))
        # coalesce with the right, then the left neighbour
        if i + 1 < len(self.free) and off + need == self.free[i + 1][0]:
            self.free[i] = (off, need + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]
        self.in_use -= need


def batch_bytes(total_keys: int, nseg: int, dtype: torch.dtype, in_place: bool, min_run: int | None = None) -> int:
    """Arena bytes of one batch: the sort's workspace for this key type,
    size and segment count, plus gathered keys and payloads unless the batch
    is sorted in place."""
    ws = binding.workspace_bytes(total_keys, nseg, dtype, True, min_run)
    if ws == 0:
        raise ValueError(f"a batch of {total_keys} keys in {nseg} segments exceeds the library's limits")
    gather = 0 if in_place else _align(total_keys * KEY_BYTES[dtype]) + _align(total_keys * 4)
    return _align(ws) + gather


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    batch: list = field(default_factory=list)
    event: torch.cuda.Event | None = None   # end of the batch on the device
    start_ev: torch.cuda.Event | None = None
    costs: torch.Tensor | None = None
    block: tuple[int, int] | None = None    # (offset, bytes) in the arena
    start_s: float = 0.0
    off_host: torch.Tensor | None = None    # pinned offsets, alive until the batch completes


class SortServer:
    """Continuous-batching sort server (one GPU, several in-flight batches)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 2, max_batch_keys: int | None = None,
                 min_run: int | None = None, max_segments: int = 4096, device="cuda"):
        binding.load_library()
        self.budget = int(hbm_budget_bytes)
        if self.budget < ALIGN:
            raise ValueError("HBM budget too small")
        self.min_run = min_run
        self.max_segments = max_segments
        self.max_batch_keys = max_batch_keys
        self.arena = torch.empty(self.budget, dtype=torch.uint8, device=device)
        self.alloc = ArenaAllocator(self.budget)
        self.slots = [_Slot(stream=torch.cuda.Stream(device=device)) for _ in range(max(slots, 1))]
        self.busy_s = 0.0
        self.stats = {}
        self.device_intervals: list[tuple[float, float]] = []

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

    def request_bytes(self, r: ServedRequest) -> int:
        """Arena bytes of a batch holding r alone (gathered unless it is a pool request)."""
        return batch_bytes(r.n, 1, r.keys.dtype, r.pool is not None, self.min_run)

    def _form(self, pending: list[ServedRequest], room: int):
        """The next batch: requests of the oldest pending request's key type,
        in arrival order, while the batch's bytes fit `room`.  A batch that
        starts with a pool request takes only the next requests of that pool
        (it stays one slice of it); others are gathered.  Returns (batch,
        rest, bytes)."""
        head = pending[0]
        dt = head.keys.dtype
        in_place = head.pool is not None
        batch, keys, need = [], 0, 0
        rest, stop = [], False
        for r in pending:
            if stop or r.keys.dtype != dt:
                rest.append(r)
                continue
            if len(batch) >= self.max_segments or (self.max_batch_keys and keys + r.n > self.max_batch_keys):
                stop = True
                rest.append(r)
                continue
            if in_place and batch:
                last = batch[-1]
                if r.pool is not last.pool or r.offset != last.offset + last.n:
                    stop = True  # later requests of that pool lie further on
                    rest.append(r)
                    continue
            b = batch_bytes(keys + r.n, len(batch) + 1, dt, in_place, self.min_run)
            if b > room:
                stop = True  # FIFO within a key type: no later request overtakes it
                rest.append(r)
                continue
            batch.append(r)
            keys += r.n
            need = b
        return batch, rest, need

    def _launch(self, slot: _Slot, batch: list[ServedRequest], block: tuple[int, int], now: float):
        dt = batch[0].keys.dtype
        kb = KEY_BYTES[dt]
        sizes = [r.n for r in batch]
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum(sizes)
        total = int(offs[-1])
        in_place = batch[0].pool is not None
        assert in_place == self._in_place(batch)
        base, nbytes = block
        ws_bytes = _align(binding.workspace_bytes(total, len(batch), dt, True, self.min_run))
        workspace = self.arena[base:base + ws_bytes]
        if in_place:
            a0 = batch[0].offset
            keys, pay = batch[0].pool.keys[a0:a0 + total], batch[0].pool.payload[a0:a0 + total]
        else:
            k0 = base + ws_bytes
            p0 = k0 + _align(total * kb)
            keys = self.arena[k0:k0 + total * kb].view(dt)
            pay = self.arena[p0:p0 + total * 4].view(torch.int32).view(torch.uint32)
        assert base + nbytes <= self.budget
        main = torch.cuda.current_stream()
        slot.stream.wait_stream(main)  # request buffers were produced on the caller's stream
        with torch.cuda.stream(slot.stream):
            start = torch.cuda.Event(enable_timing=True)
            start.record(slot.stream)
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
                                   stream=slot.stream, workspace=workspace)
            if not in_place:
                for r, a, b in zip(batch, offs[:-1], offs[1:]):
                    r.keys.copy_(keys[a:b])
                    r.payload.copy_(pay[a:b])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(slot.stream)
        slot.batch, slot.event, slot.start_ev, slot.costs, slot.start_s = batch, ev, start, costs, now
        slot.block = block
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
        self._events.append((slot.start_ev, slot.event))
        self.alloc.release(*slot.block)
        slot.batch, slot.event, slot.start_ev, slot.costs, slot.block, slot.off_host = [], None, None, None, None, None
        return True

    # --------------------------------------------------------------------- loop

    def serve(self, requests: list[ServedRequest], realtime: bool = True) -> list[ServedRequest]:
        """Serve an open-loop trace (requests sorted by arrival).  Returns the
        completed requests in completion order; latencies are done_s - arrival_s.
        With realtime=False every request is available at time 0 (saturation)
        and its arrival_s is set to 0.  Afterwards ``stats`` holds admission
        counts and ``device_intervals`` each batch's [start, end) on the
        device, in seconds from the start of the call."""
        if not realtime:
            for r in requests:
                r.arrival_s = 0.0
        for r in requests:
            if self.request_bytes(r) > self.budget:
                raise ValueError(f"request {r.rid} of {r.n} keys needs {self.request_bytes(r)} bytes, "
                                 f"more than the HBM budget of {self.budget}")
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        self._events = []
        stats = {"batches": 0, "memory_waits": 0, "max_inflight": 0, "peak_bytes": 0}
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
                batch, rest, need = self._form(pending, self.alloc.largest_free())
                if not batch:
                    # a slot is free but memory is not: wait for a batch to finish
                    stats["memory_waits"] += 1
                    break
                off = self.alloc.alloc(need)
                assert off is not None
                pending = rest
                self._launch(s, batch, (off, need), now)
                stats["batches"] += 1
                stats["max_inflight"] = max(stats["max_inflight"], sum(x.event is not None for x in self.slots))
                stats["peak_bytes"] = max(stats["peak_bytes"], self.alloc.in_use)
                progressed = True
            if not progressed:
                time.sleep(2e-5)
        torch.cuda.synchronize()
        self.device_intervals = [(ref.elapsed_time(a) / 1e3, ref.elapsed_time(b) / 1e3) for a, b in self._events]
        self._events = []
        self.stats = stats
        return done


def serve_plain(requests: list[ServedRequest], min_run: int | None = None, realtime: bool = True,
                intervals: list | None = None):
    """FIFO, one ps_sort per request on the current stream, no batching.
    realtime=False: every request is available at time 0 (arrival_s set to 0).
    intervals (a list, optional) receives each request's [start, end) on the
    device, in seconds from the start of the call."""
    if not realtime:
        for r in requests:
            r.arrival_s = 0.0
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    t0 = time.perf_counter()
    done = []
    inflight = []
    events = []
    nxt = 0
    s = torch.cuda.current_stream()
    while len(done) < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(requests) and (requests[nxt].arrival_s <= now or not realtime):
            r = requests[nxt]
            M = torch.zeros(1, dtype=torch.int64, device=r.keys.device)
            r.launch_s = now
            a = torch.cuda.Event(enable_timing=True)
            a.record(s)
            binding.sort(r.keys, r.payload, min_run=min_run, merge_cost=M)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
            events.append((a, ev))
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
    torch.cuda.synchronize()
    if intervals is not None:
        intervals.extend((ref.elapsed_time(a) / 1e3, ref.elapsed_time(b) / 1e3) for a, b in events)
    return done


def busy_time(intervals: list[tuple[float, float]]) -> float:
    """Length of the union of [start, end) intervals, e.g. (launch_s, done_s)
    of served requests: the time with work in flight."""
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


def latency_stats(done: list[ServedRequest], hbm_peak_bps: float = 8.0e12,
                  device_intervals: list[tuple[float, float]] | None = None) -> dict:
    """p50/p99/mean latency (arrival to completion), keys/s over the span, and
    the roofline fraction of the algorithmic bytes over the busy time: the
    union of the batches' device intervals when given (with their overlap,
    the summed interval lengths over that union), else the host-observed
    union of launch-to-completion intervals."""
    lat = np.array([r.done_s - r.arrival_s for r in done]) * 1e3
    keys = sum(r.n for r in done)
    span = max(r.done_s for r in done) - min(r.arrival_s for r in done)
    host_busy = busy_time([(r.launch_s, r.done_s) for r in done])
    b_alg = algorithmic_bytes(done)
    out = {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
           "keys": int(keys), "span_s": round(span, 4), "keys_per_s": round(keys / span, 1),
           "host_busy_s": round(host_busy, 4), "algorithmic_bytes": int(b_alg)}
    busy = host_busy
    if device_intervals:
        dev_busy = busy_time(device_intervals)
        work = sum(b - a for a, b in device_intervals)
        out.update({"device_busy_s": round(dev_busy, 4), "device_work_s": round(work, 4),
                    "device_overlap": round(work / dev_busy, 3) if dev_busy > 0 else None})
        busy = dev_busy
    out["busy_roofline_frac"] = round(b_alg / busy / hbm_peak_bps, 4) if busy > 0 else None
    return out
