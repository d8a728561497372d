"""Batched sorting: many arrays of uneven sizes sorted together.

A ``SegmentedBatch`` keeps one batch device-resident: the concatenated keys
and payloads, the segment offsets, per-segment merge costs and a workspace
sized by ``ps_workspace_bytes``.  ``sort()`` enqueues one
``ps_segmented_sort`` (every segment an independent powersort with its own n
and origin); ``capture()`` records that launch sequence once as a hipGraph
(through ``torch.cuda.CUDAGraph``) so that later batches of the same shape
replay it with a single graph launch.  The caller-owned workspace keeps
captured launches free of allocations.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding

_DTYPES = {np.dtype(np.int32): torch.int32, np.dtype(np.uint32): torch.uint32, np.dtype(np.int64): torch.int64,
           np.dtype(np.uint64): torch.uint64, np.dtype(np.float32): torch.float32}


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """Host array -> device tensor with the same bit patterns (unsigned types included)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).to(device).view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).to(device).view(torch.uint64)
    return torch.from_numpy(a).to(device)


class SegmentedBatch:
    """One device-resident batch sorted by ps_segmented_sort."""

    def __init__(self, offsets: np.ndarray, key_dtype, with_payload: bool = True, min_run: int | None = None,
                 device="cuda"):
        binding.load_library()
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.nseg = int(offsets.shape[0] - 1)
        self.n = int(offsets[-1])
        self.min_run = min_run
        tdt = _DTYPES[np.dtype(key_dtype)]
        self.keys = torch.empty(self.n, dtype=torch.int64 if tdt == torch.uint64 else
                                (torch.int32 if tdt == torch.uint32 else tdt), device=device)
        if tdt in (torch.uint32, torch.uint64):
            self.keys = self.keys.view(tdt)
        self.payload = torch.empty(self.n, dtype=torch.int32, device=device).view(torch.uint32) if with_payload \
            else None
        self.offsets = torch.from_numpy(offsets.view(np.int64)).to(device)
        self.costs = torch.zeros(self.nseg, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        ws = binding.workspace_bytes(self.n, self.nseg, tdt, with_payload, min_run)
        if ws == 0:
            raise ValueError("batch exceeds the library's limits")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        self.graph = None

    def load(self, keys: torch.Tensor, payload: torch.Tensor | None = None):
        """Copy a batch of the same shape into the resident buffers (device to device)."""
        self.keys.copy_(keys)
        if self.payload is not None and payload is not None:
            self.payload.copy_(payload)

    def sort(self, stream=None):
        """Enqueue one ps_segmented_sort of the resident batch."""
        binding.segmented_sort(self.keys, self.payload, self.offsets, min_run=self.min_run,
                               merge_costs=self.costs, status=self.status, stream=stream,
                               workspace=self.workspace)

    def capture(self):
        """Record sort() as a graph; the first (eager) call has already set up
        the library's one-time state, so the captured launches allocate nothing."""
        self.sort()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.sort()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
