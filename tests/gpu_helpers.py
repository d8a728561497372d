"""Helpers shared by the GPU parity tests: host<->device copies that keep the
exact bit patterns of every key type, and oracle-side reference structures."""
from __future__ import annotations

import numpy as np

_VIEW = {np.dtype(np.int32): None, np.dtype(np.uint32): np.int32, np.dtype(np.int64): None,
         np.dtype(np.uint64): np.int64, np.dtype(np.float32): None}


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32).copy()).cuda().view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).cuda().view(torch.uint64)
    return torch.from_numpy(a.copy()).cuda()


def to_host(t, dtype) -> np.ndarray:
    import torch
    dtype = np.dtype(dtype)
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    if t.dtype == torch.uint64:
        return t.view(torch.int64).cpu().numpy().view(np.uint64)
    return t.cpu().numpy().view(dtype) if t.cpu().numpy().dtype.itemsize == dtype.itemsize else t.cpu().numpy()


def merges_from_ranges(starts: np.ndarray, powers: np.ndarray, left: np.ndarray, right: np.ndarray) -> set:
    """(lo, mid, hi) of every internal node from the leaf ranges [left, right)."""
    out = set()
    r = len(starts) - 1
    for j in range(1, r):
        if powers[j] == 0:
            continue
        out.add((int(starts[left[j]]), int(starts[j]), int(starts[right[j]])))
    return out


def oracle_leaf_depths(starts: np.ndarray, merges: np.ndarray) -> np.ndarray:
    """Depth of every leaf = number of oracle merges whose range covers it."""
    r = len(starts) - 1
    d = np.zeros(r, np.int64)
    if r == 0:
        return d
    s = starts[:-1].astype(np.int64)
    for lo, _, hi in merges.astype(np.int64):
        a = np.searchsorted(s, lo, side="left")
        b = np.searchsorted(s, hi, side="left")
        d[a:b] += 1
    return d
