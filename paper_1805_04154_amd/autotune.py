"""Autotuner for the launch shape of the data-movement kernels.

The tunables (``ps_tuning``) change speed only, never results: the number of
merge-tree levels one merge pass does (1, or 2 with absorbed children), the
grid sizes of the grid-stride kernels and the merge-path tile (2048, 4096 or
8192 outputs).
``tune()`` times every candidate on a caller-supplied step (which must
restore its own input before sorting), keeps the fastest, and records it in a
JSON cache keyed by a workload signature so later runs start from the tuned
shape.  Timing uses HIP events on the current stream around the sort only.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import binding

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "powersort_hip", "tuning.json")
# Shapes measured on an MI355X and shipped with the package: consulted after
# the user's cache, so that a run without a tuning pass starts from a tuned
# shape (written by tune() + save_cache(..., path=SHIPPED_CACHE)).
SHIPPED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def candidates(small: bool = False) -> list[dict]:
    """The search space: tree levels per merge pass (1, or 2 with absorbed
    children) x merge tile x merge grid x fused grid x split grid."""
    levels = (1, 2)
    tiles = (8192, 4096, 2048)
    merge_grids = (1024, 2048, 4096) if not small else (2048,)
    fused_grids = (2048, 4096, 8192) if not small else (2048,)
    split_grids = (1024, 2048, 4096) if not small else (2048,)
    out = []
    for lv, t, gm, gf, gs in itertools.product(levels, tiles, merge_grids, fused_grids, split_grids):
        out.append({"merge_levels": lv, "merge_tile": t, "grid_merge": gm, "grid_fused": gf, "grid_split": gs,
                    "grid_big_leaf": 2048})
    return out


def signature(n_total: int, nseg: int, dtype: torch.dtype, min_run: int | None, kind: str = "") -> str:
    """Workload signature: sizes are bucketed to powers of two."""
    lg = max(0, int(n_total).bit_length() - 1)
    ls = max(0, int(nseg).bit_length() - 1)
    return f"{kind}n2^{lg}_seg2^{ls}_{str(dtype).replace('torch.', '')}_w{min_run or 24}"


def time_step(restore, step, reps: int = 3) -> float:
    """Median milliseconds of step() over reps runs, restore() before each (untimed)."""
    ts = []
    s = torch.cuda.current_stream()
    for _ in range(reps):
        restore()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        step()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(restore, step, cands: list[dict] | None = None, reps: int = 3, verbose: bool = False) -> tuple[dict, list]:
    """Time every candidate; leave the best one set and return it with all timings."""
    cands = cands if cands is not None else candidates()
    before = binding.get_tuning()
    results = []
    try:
        for c in cands:
            binding.set_tuning(c)
            step()  # warm-up at this shape
            torch.cuda.synchronize()
            ms = time_step(restore, step, reps)
            results.append((ms, c))
            if verbose:
                print(f"  {ms:8.3f} ms  {c}", flush=True)
    except Exception:
        binding.set_tuning(before)
        raise
    results.sort(key=lambda x: x[0])
    best = results[0][1]
    binding.set_tuning(best)
    return best, results


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(key: str, tuning: dict, ms: float, path: str = DEFAULT_CACHE):
    data = load_cache(path)
    data[key] = {"tuning": tuning, "ms": ms}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str, paths=(DEFAULT_CACHE, SHIPPED_CACHE)) -> dict | None:
    """The cached shape for a signature: the first cache that holds it
    (paths: one cache file or a sequence of them)."""
    if isinstance(paths, (str, os.PathLike)):
        paths = (paths,)
    for path in paths:
        entry = load_cache(path).get(key)
        if entry:
            return entry["tuning"]
    return None


def apply_cached(key: str, paths=(DEFAULT_CACHE, SHIPPED_CACHE)) -> dict | None:
    """Set the cached shape for a signature, if one exists."""
    tuning = lookup(key, paths)
    if tuning:
        binding.set_tuning(tuning)
    return tuning
