#!/usr/bin/env python3
"""Benchmark of the MI355X powersort.

Default run (the headline and the rest of the metric, one JSON line):

* headline: one step = one ps_sort of the whole input (run detection, leaf
  partition, node powers, merge tree, leaf formation and every merge) on a
  fresh copy of the input already resident in HBM.  n = 2^28 int32 keys with
  a uint32 index payload, runs of Zipf(1.2) lengths (clipped to 2^24), keys
  uniform in [0, 2^20), 10% strictly descending runs.  Reports keys/s, the
  HBM roofline of the merge-pass kernel (HIP dispatch events of the timed
  region; the committed rocprofv3 trace's duration beside it), the whole-path
  fraction of the roofline from the merge cost, and the CPU oracle on the same
  input as a reported baseline (one pinned host core, one warm-up, three
  timed calls, median; its merge cost must equal the GPU's);
* ``latency_2p20``: per-sort latency (p50/p99) of one 2^20-key sort (runs of
  lengths uniform in [1, 2048]), launched eagerly and as a replayed hipGraph;
* ``batched``: 4096 arrays of log-uniform sizes in [2^10, 2^22] sorted by one
  ps_segmented_sort (eager and as a replayed graph, launch shape from the
  shipped tuning cache) against 4096 plain ps_sort calls;
* ``served``: a Poisson trace of sort requests served by the continuous-
  batching server and by plain per-request calls, open loop and saturated:
  p50/p99 latency, keys/s, device busy time and overlap of batches.

``--headline-only`` prints the headline alone; ``--workload`` selects other
single workloads (see WORKLOADS).

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E
METRIC = "keys/s and % HBM roofline (2^28 int32+idx); batched/served vs plain; p50/p99"
WORKLOADS = ("zipf_i32", "zipf_u64", "perm_i32", "runs_i32", "runs_2p20", "batched", "served", "alphabetic",
             "mergecost")
MERGECOST_METRIC = ("merge cost M/n of powersort and peeksort (GPU ps_merge_cost) against the entropy bound and "
                    "the paper's top-down and bottom-up mergesorts (oracle), per input family; merge-cost keys/s")
ALPHA_METRIC = "alphabetic tree (Method 2') leaves/s: node powers, tree, depths and weighted path length"
SERVED_METRIC = ("served sorts: p50/p99 latency and keys/s, continuous batching vs plain per-request calls "
                 "(Poisson 2000 req/s, sizes 2^12..2^24, int32/int64/float32 keys + uint32 payload)")
BATCHED_METRIC = "batched segmented sort keys/s vs plain per-array calls (4096 arrays, log-uniform sizes 2^10..2^22)"
LATENCY_METRIC = "single-sort latency p50/p99 (2^20 int32 keys + uint32 index, runs U[1,2048]), eager and hipGraph"


def make_workload(name: str, n: int):
    from paper_1805_04154_amd import workloads as W
    if name == "zipf_i32":
        return W.zipf_runs(n, key_dtype=np.int32)
    if name == "zipf_u64":
        return W.zipf_runs(n, key_dtype=np.uint64)
    if name == "perm_i32":
        return W.permutation_i32(n)
    if name == "runs_i32":
        return W.runs_sqrt_i32(n)
    raise ValueError(name)


def to_dev(a: np.ndarray):
    import torch
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda().view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda().view(torch.uint64)
    return torch.from_numpy(a).cuda()


COUNTERS_MD = os.path.join(ROOT, "profiles", "merge_pass_counters_zipf_2p28_i32.md")
TRACE_MD = os.path.join(ROOT, "profiles", "kernels_zipf_2p28_i32.md")


def merge_kernel_digest() -> str:
    """Digest of the source text of the kernel the roofline measures, the
    two-input merge pass (its body, its LDS padding and its sample writes)."""
    src = open(os.path.join(ROOT, "paper_1805_04154_amd", "csrc", "merge.hip")).read()
    a = src.index("__device__ __forceinline__ uint32_t lpad(")
    parts = [src[a:src.index("\n", a)]]  # the one-line padding function
    for start in ("void merge_pass_kernel(MoveArgs a, uint32_t p) {", "void put_samples_lds("):
        a = src.index(start)
        parts.append(src[a:src.index("\n}\n", a)])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def profile_fields(path: str) -> dict:
    """The machine-readable "- key: `value`" lines of a committed profile summary."""
    fields = {}
    try:
        text = open(path).read()
    except OSError:
        return fields
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    return fields


def measured_traffic(workload: str, launches_per_sort: int, merge_tile: int):
    """HBM bytes per merge-pass launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a device copy), if
    it was taken on this workload, on the current kernel source, with the
    same merge tile and number of merge launches per sort; else None."""
    fields = profile_fields(COUNTERS_MD)
    if fields.get("workload") != workload or fields.get("kernel_source_digest") != merge_kernel_digest():
        return None
    if fields.get("merge_launches_per_sort") != str(launches_per_sort):
        return None
    if fields.get("merge_tile") != str(merge_tile):
        return None
    try:
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def traced_launch_ms(workload: str, merge_tile: int):
    """Average merge-pass duration (ms) in the committed rocprofv3 kernel
    trace of this workload, if it was taken on the current kernel source with
    the same merge tile; else None."""
    fields = profile_fields(TRACE_MD)
    if fields.get("workload") != workload or fields.get("kernel_source_digest") != merge_kernel_digest():
        return None
    if fields.get("merge_tile") != str(merge_tile):
        return None
    try:
        return float(fields["merge_pass_average_ns"]) / 1e6
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------ CPU baselines

def host_cpu() -> str:
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def usable_cores() -> list[int]:
    """Cores this process may run on, at most 16 (one GPU's share of a box)."""
    try:
        cores = sorted(os.sched_getaffinity(0))
    except AttributeError:
        cores = list(range(os.cpu_count() or 1))
    return cores[-16:]


def host_cores() -> int:
    return max(1, len(usable_cores()))


def run_pinned(fn, core: int | None = None):
    """fn() in a new thread bound to one host core (sched_setaffinity of the
    calling thread); the GPU runtime's threads are not affected.  Returns
    (fn's result, the core)."""
    core = usable_cores()[-1] if core is None else core
    box = {}

    def body():
        try:
            os.sched_setaffinity(0, {core})
            box["r"] = fn()
        except BaseException as e:  # re-raised in the caller
            box["e"] = e

    t = threading.Thread(target=body)
    t.start()
    t.join()
    if "e" in box:
        raise box["e"]
    return box["r"], core


def oracle_timing(sort, keys, payload, reps: int, warmup: int = 1):
    """One warm-up call and `reps` timed calls of the oracle on the same
    input, on a pinned core: (median seconds, all seconds, merge costs, core)."""
    def work():
        for _ in range(warmup):
            sort(keys, payload, details=False)
        ts, ms = [], []
        for _ in range(reps):
            t = time.perf_counter()
            r = sort(keys, payload, details=False)
            ts.append(time.perf_counter() - t)
            ms.append(int(r.merge_cost))
        return ts, ms
    (ts, ms), core = run_pinned(work)
    return float(np.median(ts)), ts, ms, core


def cpu_baseline(wl, method: str = "powersort", reps: int = 3) -> dict:
    """The oracle as it stands on the whole workload: one pinned host core,
    one warm-up call, `reps` timed calls, the median.  Its merge cost is
    returned for the caller to compare with the GPU's."""
    import oracle
    sort = oracle.powersort if method == "powersort" else oracle.peeksort
    med, ts, ms, core = oracle_timing(sort, wl.keys, wl.payload, reps)
    return {"value": round(wl.n / med, 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "median_s": round(med, 3), "times_s": [round(t, 3) for t in ts], "merge_cost": ms[0],
            "merge_costs_agree": len(set(ms)) == 1,
            "sample": f"all {wl.n} keys of the same workload (payload = index), one {method} call per rep: "
                      f"1 warm-up + {reps} timed, median; one thread pinned to host core {core} "
                      f"({host_cpu()}, {os.cpu_count()} logical cores visible)"}


def batched_cpu_baseline(wl, budget_s: float) -> dict:
    """The oracle on the batch's segments, each an independent powersort: one
    pinned core in segment order for budget_s / 2 (after one warm-up call on
    segment 0), then every usable core (one thread pinned to each; the C
    oracle runs without the GIL) on the following segments for as long.
    Segment sizes are i.i.d., so either prefix is a fair sample."""
    import oracle
    offs = wl.offsets.astype(np.int64)
    nseg = offs.shape[0] - 1

    def one(i):
        a, b = int(offs[i]), int(offs[i + 1])
        oracle.powersort(wl.keys[a:b], wl.payload[a:b], details=False)
        return b - a

    def serial():
        one(0)  # warm-up
        t0 = time.perf_counter()
        k1, i = 0, 0
        while i < nseg and time.perf_counter() - t0 < budget_s / 2:
            k1 += one(i)
            i += 1
        return k1, i, time.perf_counter() - t0

    (k1, first_all, dt1), core = run_pinned(serial)
    cores = usable_cores()
    lock = threading.Lock()
    state = {"next": first_all, "keys": 0}
    t0 = time.perf_counter()

    def worker(c):
        os.sched_setaffinity(0, {c})
        while True:
            with lock:
                if state["next"] >= nseg or time.perf_counter() - t0 >= budget_s / 2:
                    return
                j = state["next"]
                state["next"] += 1
            kk = one(j)
            with lock:
                state["keys"] += kk

    threads = [threading.Thread(target=worker, args=(c,)) for c in cores]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dt_all = time.perf_counter() - t0
    return {"value": round(k1 / dt1, 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"segments 0..{first_all - 1} of {nseg} ({k1} keys), one oracle powersort per segment "
                      f"after one warm-up call, one thread pinned to host core {core} ({host_cpu()}), {dt1:.2f} s",
            "all_cores": {"value": round(state["keys"] / dt_all, 1), "unit": "keys/s", "cores": len(cores),
                          "sample": f"segments {first_all}..{state['next'] - 1} ({state['keys']} keys), "
                                    f"{len(cores)} threads, each pinned to its own core, running oracle calls "
                                    f"on whole segments, {dt_all:.2f} s"}}


def served_cpu_baseline(keys_list, budget_s: float) -> dict:
    """Single-core oracle service time per request, over the trace's first
    requests until budget_s (after one warm-up call on the first): p50/p99
    of one oracle powersort call each, on a pinned core."""
    import oracle
    from paper_1805_04154_amd import workloads as W

    def work():
        oracle.powersort(keys_list[0], W.payload_for(len(keys_list[0])), details=False)
        ts, nk = [], 0
        t0 = time.perf_counter()
        for k in keys_list:
            if time.perf_counter() - t0 >= budget_s:
                break
            pay = W.payload_for(len(k))
            t = time.perf_counter()
            oracle.powersort(k, pay, details=False)
            ts.append(time.perf_counter() - t)
            nk += len(k)
        return ts, nk

    (ts, nk), core = run_pinned(work)
    a = np.asarray(ts) * 1e3
    return {"value": round(float(nk / (a.sum() / 1e3)), 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "service_ms": {"p50": round(float(np.percentile(a, 50)), 3), "p99": round(float(np.percentile(a, 99)), 3)},
            "sample": f"first {len(ts)} requests of the trace ({nk} keys), one oracle powersort call each after "
                      f"one warm-up call, one thread pinned to host core {core} ({host_cpu()})"}


def percentiles_ms(samples_s) -> dict:
    """Median, p10 and p90 of per-sort durations, in ms."""
    a = np.sort(np.asarray(samples_s, dtype=np.float64)) * 1e3
    return {"median": round(float(np.median(a)), 4), "p10": round(float(np.percentile(a, 10)), 4),
            "p90": round(float(np.percentile(a, 90)), 4), "sorts": int(a.size)}


def latency_ms(samples_s) -> dict:
    """p50/p99/mean/min/max of per-sort durations, in ms."""
    a = np.asarray(samples_s, dtype=np.float64) * 1e3
    return {"p50": round(float(np.percentile(a, 50)), 4), "p99": round(float(np.percentile(a, 99)), 4),
            "mean": round(float(a.mean()), 4), "min": round(float(a.min()), 4), "max": round(float(a.max()), 4),
            "sorts": int(a.size)}


def free_device_memory():
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# --------------------------------------------------------------- headline

def run_headline(args):
    """The plain sort of one array (default: the 2^28 Zipf-runs headline).
    Returns (the JSON line without cpu_baseline, the workload) or (error, None)."""
    import torch
    from paper_1805_04154_amd import binding

    binding.load_library()
    binding.set_tuning(None)
    n = 1 << args.log2n
    t_gen = time.perf_counter()
    wl = make_workload(args.workload, n)
    t_gen = time.perf_counter() - t_gen
    kb = wl.keys.dtype.itemsize
    rec_bytes = kb + 4  # key + uint32 payload

    # Fresh copies of the input for every step, staged in HBM before timing.
    src_k, src_p = to_dev(wl.keys), to_dev(wl.payload)
    copies = [(src_k.clone(), src_p.clone()) for _ in range(args.steps)]
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def refill():
        for k, p in copies:
            k.copy_(src_k)
            p.copy_(src_p)
        torch.cuda.synchronize()

    def region(groups, per_sort=False):
        """Sort every copy back to back; groups: kernel groups timed with
        HIP events on the sort's stream (None: no events at all).  With
        per_sort, an event between consecutive sorts gives each one's
        duration (returned in place of the total)."""
        refill()
        binding.profile_enable(groups is not None, groups=groups if groups else None)
        binding.profile_read(reset=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(copies) + 1 if per_sort else 2)]
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        ev[0].record(stream)
        for i, (k, p) in enumerate(copies):
            binding.sort(k, p, min_run=args.min_run, merge_cost=M, method=args.method)
            if per_sort:
                ev[i + 1].record(stream)
        ev[-1].record(stream)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        pr = binding.profile_read(reset=True) if groups is not None else None
        binding.profile_enable(False)
        if per_sort:
            return t_b - t_a, [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(len(copies))], pr
        return t_b - t_a, ev[0].elapsed_time(ev[-1]) / 1e3, pr

    for i in range(args.warmup):
        k, p = copies[i % len(copies)]
        k.copy_(src_k)
        p.copy_(src_p)
        binding.sort(k, p, min_run=args.min_run, merge_cost=M, method=args.method)
    torch.cuda.synchronize()

    # Timed region: every merge-pass launch carries its own dispatch events.
    wall_s, ev_s, prof = region(("merge",))
    # Verify the timed region's last step before anything overwrites it.
    k_out, p_out = copies[-1]
    kh = k_out.view(torch.int64 if kb == 8 else torch.int32).cpu().numpy()
    ph = p_out.view(torch.int32).cpu().numpy().view(np.uint32)
    # Informational: the same steps without any events, and with every group timed.
    plain_s, _, _ = region(None)
    _, _, prof_all = region(tuple(binding.PROF_GROUPS))
    _, per_sort_s, _ = region(None, per_sort=True)
    step_s = wall_s / args.steps
    merge_cost = int(M.item())

    # Verify the timed region's last step against properties that fix the stable sort.
    okeys = wl.keys.view(np.int64 if kb == 8 else np.int32)
    sorted_ok = bool(np.all(wl.keys[ph][1:] >= wl.keys[ph][:-1]))
    seen = np.zeros(n, dtype=bool)
    seen[ph] = True
    perm_ok = bool(seen.all())
    keys_ok = bool(np.array_equal(kh, okeys[ph]))
    eq = wl.keys[ph][1:] == wl.keys[ph][:-1]
    stable_ok = bool(np.all(ph[1:][eq] > ph[:-1][eq]))
    del seen, eq, kh, ph
    if not (sorted_ok and perm_ok and keys_ok and stable_ok):
        return {"error": "output is not the stable sort", "sorted": sorted_ok, "perm": perm_ok,
                "keys": keys_ok, "stable": stable_ok}, None

    if args.calib_copy_mib:
        a = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # Roofline of the dominant kernel: the merge-path pass.  Algorithmic bytes
    # per merged output element = read both inputs + write the result.
    # Durations: the dispatch events of every merge-pass launch of the timed
    # region.
    mp = prof["merge"]
    mp_launch_ms = mp["ms"] / max(mp["launches"], 1)
    mp_bytes = 2 * rec_bytes * mp["elems"]
    mp_bytes_per_launch = mp_bytes / max(mp["launches"], 1)
    achieved_gbs = (mp_bytes_per_launch / (mp_launch_ms / 1e3)) / 1e9 if mp_launch_ms > 0 else 0.0
    peak_gbs = HBM_PEAK_BPS / 1e9
    launches_per_sort = mp["launches"] // max(args.steps, 1)
    # 8192-output tiles apply to 4-byte keys only; 8-byte keys merge with
    # 4096-output tiles in the kernel that finds its own co-ranks
    merge_tile = binding.get_tuning()["merge_tile"]
    if kb == 8:
        merge_tile = min(merge_tile, 4096)
    same_setup = args.min_run == 24 and args.method == "powersort"
    traffic = measured_traffic(wl.name, launches_per_sort, merge_tile) if same_setup else None
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": peak_gbs, "unit": "GB/s",
                "frac": round(achieved_gbs / peak_gbs, 4), "traffic": traffic,
                "kernel": "merge_pass_kernel" if kb == 4 else "merge_pass_cr_kernel",
                "merge_tile": merge_tile, "launch_ms": round(mp_launch_ms, 4), "launches_per_sort": launches_per_sort,
                "algorithmic_bytes_per_launch": int(mp_bytes_per_launch)}
    t_ms = traced_launch_ms(wl.name, merge_tile) if same_setup else None
    if t_ms:
        # the same kernel's average duration in the committed rocprofv3 trace
        roofline["trace"] = {"launch_ms": round(t_ms, 4),
                             "frac": round(mp_bytes_per_launch / (t_ms / 1e3) / HBM_PEAK_BPS, 4),
                             "trace_over_events": round(t_ms / mp_launch_ms, 4) if mp_launch_ms > 0 else None,
                             "source": os.path.relpath(TRACE_MD, ROOT)}
    # Whole path: B_alg = (K+V)(2M + 2n) per sort, from the merge cost.
    b_alg = rec_bytes * (2 * merge_cost + 2 * n)
    path = {"algorithmic_bytes": int(b_alg), "achieved_GBps": round(b_alg / step_s / 1e9, 1),
            "frac": round(b_alg / step_s / HBM_PEAK_BPS, 4)}
    # Informational breakdown from the region with every group timed (its
    # events add some microseconds per group, so its total is not the headline).
    groups = {g: {"ms_per_step": round(prof_all[g]["ms"] / args.steps, 4),
                  "launches_per_step": prof_all[g]["launches"] // max(args.steps, 1),
                  "elems_per_step": prof_all[g]["elems"] // max(args.steps, 1)}
              for g in binding.PROF_GROUPS}

    out = {
        "metric": METRIC,
        "value": round(n * args.steps / wall_s, 1),
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"int32": "int32", "int64": "int64", "uint64": "u64", "float32": "f32"}[str(wl.keys.dtype)],
        "data": "synthetic",
        "config": {"workload": wl.name if args.method == "powersort" else f"{wl.name}_peeksort", "n": n,
                   "method": args.method, "key": str(wl.keys.dtype), "payload": "uint32 index",
                   "min_run": args.min_run, "merge_cost": merge_cost, "merge_cost_per_key": round(merge_cost / n, 4),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "path_roofline": path,
        "kernel_groups": groups,
        "event_ms_per_step": round(ev_s / args.steps * 1e3, 4),
        "ms_per_step_without_events": round(plain_s / args.steps * 1e3, 4),
        "per_sort_ms": percentiles_ms(per_sort_s),
        "gen_s": round(t_gen, 2),
    }
    del copies, src_k, src_p, k_out, p_out
    free_device_memory()
    return out, wl


# ------------------------------------------------------- single-sort latency

def run_latency(args, reps: int = 200, cpu: bool = True) -> dict:
    """Latency of one 2^20-key sort (runs of lengths uniform in [1, 2048],
    keys in [0, 2^16), 25% strictly descending; int32 + uint32 index):
    `reps` sorts, each from a freshly restored input (outside its events),
    launched eagerly and as one replayed hipGraph of the same sort (captured
    with a caller workspace, so the captured launches allocate nothing).
    Both results are checked against the oracle."""
    import torch
    import oracle
    from paper_1805_04154_amd import binding, workloads as W

    binding.load_library()
    binding.set_tuning(None)
    n = 1 << 20
    wl = W.runs_2p20(n)
    src_k, src_p = to_dev(wl.keys), to_dev(wl.payload)
    k, p = src_k.clone(), src_p.clone()
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(binding.workspace_bytes(n, 1, torch.int32, True, args.min_run), dtype=torch.uint8,
                     device="cuda")
    s = torch.cuda.current_stream()

    def restore():
        k.copy_(src_k)
        p.copy_(src_p)

    def eager():
        binding.sort(k, p, min_run=args.min_run, merge_cost=M, workspace=ws)

    def timed(step):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            restore()
            a.record(s)
            step()
            b.record(s)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) / 1e3 for a, b in evs]

    ref = oracle.powersort(wl.keys, wl.payload, min_run=args.min_run, details=False)

    def matches() -> bool:
        torch.cuda.synchronize()
        return (np.array_equal(k.cpu().numpy(), ref.keys)
                and np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), ref.payload)
                and int(M.item()) == ref.merge_cost)

    for _ in range(10):
        restore()
        eager()
    torch.cuda.synchronize()
    t_eager = timed(eager)
    ok_eager = matches()
    # kernel launches of one sort: the profiled groups plus the offsets,
    # counter-initialisation and merge-cost copy kernels
    binding.profile_enable(True)
    binding.profile_read(reset=True)
    restore()
    eager()
    pr = binding.profile_read(reset=True)
    binding.profile_enable(False)
    launches = sum(pr[g]["launches"] for g in binding.PROF_GROUPS) + 3
    g = torch.cuda.CUDAGraph()
    restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        eager()
    torch.cuda.synchronize()
    for _ in range(5):
        restore()
        g.replay()
    t_graph = timed(g.replay)
    ok_graph = matches()
    if not (ok_eager and ok_graph):
        return {"error": "2^20-key sort differs from the oracle", "eager": ok_eager, "graph": ok_graph}
    b_alg = 8 * (2 * ref.merge_cost + 2 * n)
    e, gr = latency_ms(t_eager), latency_ms(t_graph)
    out = {"metric": LATENCY_METRIC, "value": round(n / (gr["p50"] / 1e3), 1), "unit": "keys/s",
           "workload": wl.name, "n": n, "merge_cost": ref.merge_cost, "kernel_launches_per_sort": launches,
           "eager_ms": e, "graph_ms": gr,
           "keys_per_s_eager_p50": round(n / (e["p50"] / 1e3), 1),
           "path_roofline_frac_graph_p50": round(b_alg / (gr["p50"] / 1e3) / HBM_PEAK_BPS, 4),
           "checked_against_oracle": True,
           "note": "the 12 MB input and scratch fit the 256 MB Infinity Cache; latency-bound, not a roofline case"}
    if cpu:
        med, ts, ms, core = oracle_timing(oracle.powersort, wl.keys, wl.payload, reps=10)
        out["cpu_baseline"] = {"value": round(n / med, 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
                               "median_ms": round(med * 1e3, 3),
                               "sample": f"the same {n} keys, 1 warm-up + 10 timed oracle calls, median; one "
                                         f"thread pinned to host core {core} ({host_cpu()})"}
    del src_k, src_p, k, p, ws, g
    free_device_memory()
    return out


# -------------------------------------------------------------------- batched

def run_batched(args, cpu: bool = True) -> dict:
    """4096 arrays of log-uniform sizes: plain per-array ps_sort calls vs one
    ps_segmented_sort (eager and replayed as a captured hipGraph) under the
    launch shape of the tuning cache (the autotuner runs only with --tune).
    Every timed sort starts from the same unsorted input, restored outside
    the timed region."""
    import torch
    from paper_1805_04154_amd import autotune, batched, binding, workloads as W

    binding.load_library()
    binding.set_tuning(None)
    t_gen = time.perf_counter()
    wl = W.batched_random_runs(nseg=args.segments)
    t_gen = time.perf_counter() - t_gen
    n, nseg = wl.n, args.segments
    offs = wl.offsets.astype(np.int64)
    src_k = batched.to_device(wl.keys)
    src_p = batched.to_device(wl.payload)
    b = batched.SegmentedBatch(wl.offsets, wl.keys.dtype, min_run=args.min_run)
    s = torch.cuda.current_stream()
    reps = max(3, args.batched_reps)

    def restore():
        b.load(src_k, src_p)

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            restore()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2], ts

    def plain():
        for g in range(nseg):
            a, c = int(offs[g]), int(offs[g + 1])
            binding.sort(b.keys[a:c], b.payload[a:c], min_run=args.min_run)

    plain()  # warm-up (grows the per-stream pool to the largest array)
    torch.cuda.synchronize()
    plain_ms, _ = timed(plain, 3)
    key = autotune.signature(n, nseg, torch.int32, args.min_run, "batched_")
    if args.tune:
        tuned, results = autotune.tune(restore, b.sort, autotune.candidates(), reps=2)
        autotune.save_cache(key, tuned, results[0][0])
        source = "autotuned in this run"
    else:
        tuned = autotune.apply_cached(key)
        source = "tuning cache" if tuned else "library defaults (no cached shape for this signature)"
    b.sort()
    torch.cuda.synchronize()
    eager_ms, eager_all = timed(b.sort, reps)
    restore()
    b.capture()
    graph_ms, graph_all = timed(b.replay, reps)
    # correctness of the last replay: per segment sorted, stable, a permutation
    restore()
    b.replay()
    torch.cuda.synchronize()
    kh = b.keys.cpu().numpy()
    ph = b.payload.view(torch.int32).cpu().numpy().view(np.uint32)
    seg_of = np.repeat(np.arange(nseg, dtype=np.int32), np.diff(offs))
    ok = bool(np.array_equal(seg_of[ph], seg_of)) and bool(np.array_equal(kh, wl.keys[ph]))
    same = (seg_of[1:] == seg_of[:-1])
    del seg_of
    ok = ok and bool(np.all(kh[1:][same] >= kh[:-1][same]))
    eq = same & (kh[1:] == kh[:-1])
    ok = ok and bool(np.all(ph[1:][eq] > ph[:-1][eq]))
    del kh, ph, same, eq
    if not ok:
        return {"error": "batched output is not the per-segment stable sort"}
    M = int(b.costs.cpu().numpy().view(np.uint64).sum())
    b_alg = 8 * (2 * M + 2 * n)
    binding.profile_enable(True, groups=("merge",))
    binding.profile_read(reset=True)
    restore()
    torch.cuda.synchronize()
    b.sort()
    torch.cuda.synchronize()
    prof = binding.profile_read(reset=True)
    binding.profile_enable(False)
    mp = prof["merge"]
    mp_ms = mp["ms"] / max(mp["launches"], 1)
    ach = (2 * 8 * mp["elems"] / max(mp["launches"], 1)) / (mp_ms / 1e3) / 1e9 if mp_ms > 0 else 0.0
    best_ms = min(eager_ms, graph_ms)
    # informational: every group of one eager sort timed
    binding.profile_enable(True)
    binding.profile_read(reset=True)
    restore()
    torch.cuda.synchronize()
    b.sort()
    torch.cuda.synchronize()
    prof_all = binding.profile_read(reset=True)
    binding.profile_enable(False)
    groups = {g: round(prof_all[g]["ms"], 3) for g in binding.PROF_GROUPS}
    launches = sum(prof_all[g]["launches"] for g in binding.PROF_GROUPS) + 3
    out = {
        "metric": BATCHED_METRIC,
        "value": round(n / (graph_ms / 1e3), 1),
        "unit": "keys/s",
        "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(graph_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "segments": nseg, "key": "int32", "payload": "uint32 index",
                   "min_run": args.min_run, "merge_cost": M, "tuning": binding.get_tuning(), "tuning_source": source,
                   "signature": key},
        "plain": {"ms": round(plain_ms, 3), "keys_per_s": round(n / (plain_ms / 1e3), 1), "calls": nseg},
        "batched_eager": {"ms": round(eager_ms, 3), "keys_per_s": round(n / (eager_ms / 1e3), 1),
                          "all_ms": [round(x, 3) for x in eager_all]},
        "batched_graph": {"ms": round(graph_ms, 3), "keys_per_s": round(n / (graph_ms / 1e3), 1),
                          "all_ms": [round(x, 3) for x in graph_all]},
        "kernel_launches_per_batch": launches,
        "speedup_vs_plain": round(plain_ms / best_ms, 2),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_BPS / 1e9, "unit": "GB/s",
                     "frac": round(ach / (HBM_PEAK_BPS / 1e9), 4), "traffic": None, "kernel": "merge_pass_kernel",
                     "launch_ms": round(mp_ms, 4)},
        "path_roofline": {"algorithmic_bytes": b_alg, "frac": round(b_alg / (best_ms / 1e3) / HBM_PEAK_BPS, 4),
                          "frac_plain": round(b_alg / (plain_ms / 1e3) / HBM_PEAK_BPS, 4)},
        "kernel_groups_ms": groups,
        "gen_s": round(t_gen, 1),
    }
    binding.set_tuning(None)
    del b, src_k, src_p
    free_device_memory()
    if cpu:
        out["cpu_baseline"] = batched_cpu_baseline(wl, args.cpu_budget)
    return out


# --------------------------------------------------------------------- served

def run_served(args, cpu: bool = True) -> dict:
    """Open-loop Poisson trace served by the continuous-batching server and,
    for comparison, FIFO with one ps_sort per request; then both saturated
    (every request available at t = 0).  Inputs are device-resident."""
    import torch
    from paper_1805_04154_amd import batched, serving, workloads as W

    t_gen = time.perf_counter()
    metas = W.trace_meta(rate_hz=args.rate, duration_s=args.duration)
    keys = W.materialize(metas)
    t_gen = time.perf_counter() - t_gen
    src = [(batched.to_device(k), batched.to_device(W.payload_for(m.n))) for m, k in zip(metas, keys)]
    torch.cuda.synchronize()

    # Request buffers come from one pool per key type, in arrival order, so
    # the server sorts each batch in place; refilled from src before every
    # run (outside the served time).
    need = {}
    for k, _ in src:
        need[k.dtype] = need.get(k.dtype, 0) + k.numel()
    pools = {dt: serving.RequestPool(dt, cnt) for dt, cnt in need.items()}

    def fresh():
        for pool in pools.values():
            pool.reset()
        reqs = []
        for i, (m, (k, p)) in enumerate(zip(metas, src)):
            r = pools[k.dtype].request(i, m.arrival_s, k.numel())
            r.keys.copy_(k)
            r.payload.copy_(p)
            reqs.append(r)
        torch.cuda.synchronize()
        return reqs

    budget = int(args.budget_gib * (1 << 30))
    srv = serving.SortServer(hbm_budget_bytes=budget, slots=args.slots, min_run=args.min_run)
    # warm-up: one small batch per key type through the server and the plain path
    warm = fresh()[:6]
    for r in warm:
        r.arrival_s = 0.0
    srv.serve(warm, realtime=False)
    serving.serve_plain(fresh()[:6], min_run=args.min_run, realtime=False)

    out_runs = {}
    for name, realtime in (("open_loop", True), ("saturated", False)):
        reqs = fresh()
        done = srv.serve(reqs, realtime=realtime)
        out_runs[f"batched_{name}"] = {**serving.latency_stats(done, device_intervals=srv.device_intervals),
                                       **{f"admission_{k}": v for k, v in srv.stats.items()}}
        if name == "saturated":
            # results of the saturated batched run: per-request stable sort
            for r in done[:: max(1, len(done) // 16)]:
                kh = r.keys.cpu().numpy().view(keys[r.rid].dtype)
                ph = r.payload.view(torch.int32).cpu().numpy().view(np.uint32)
                if not np.array_equal(kh.view(np.uint8), keys[r.rid][ph].view(np.uint8)):
                    return {"error": "served output is not a permutation of the request"}
        reqs = fresh()
        iv = []
        done = serving.serve_plain(reqs, min_run=args.min_run, realtime=realtime, intervals=iv)
        out_runs[f"plain_{name}"] = serving.latency_stats(done, device_intervals=iv)
    total_keys = sum(m.n for m in metas)
    sat = out_runs["batched_saturated"]
    out = {
        "metric": SERVED_METRIC,
        "value": sat["keys_per_s"],
        "unit": "keys/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(sat["span_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/int64/float32", "data": "synthetic",
        "config": {"workload": f"poisson_{int(args.rate)}hz_{args.duration}s_logu12-24", "requests": len(metas),
                   "keys": total_keys, "slots": args.slots, "hbm_budget_gib": args.budget_gib,
                   "min_run": args.min_run, "inputs": "device-resident, one pool per key type"},
        "served": out_runs,
        "p50_ms": out_runs["batched_open_loop"]["p50_ms"],
        "p99_ms": out_runs["batched_open_loop"]["p99_ms"],
        "saturated_speedup_vs_plain": round(sat["keys_per_s"] / out_runs["plain_saturated"]["keys_per_s"], 2),
        "gen_s": round(t_gen, 1),
    }
    del srv, pools, src
    free_device_memory()
    if cpu:
        out["cpu_baseline"] = served_cpu_baseline(keys, args.cpu_budget)
    return out


def run_alphabetic(args) -> int:
    """ps_alphabetic_tree on 2^log2n leaf weights (log2n capped at 24) drawn
    as Zipf(1.2) clipped to 2^7 (heavy-tailed run lengths whose sum stays below
    2^31 at 2^24 leaves); timed over
    --steps calls with the weights resident in HBM.  The cpu_baseline leg
    times the oracle (the merge order of runs of those lengths) on the same
    weights, and the last call's output is checked against that result."""
    import torch
    from paper_1805_04154_amd import binding, workloads as W

    binding.load_library()
    r = 1 << min(args.log2n, 24)
    rng = W.config_rng(6)
    w_np = np.minimum(rng.zipf(1.2, size=r), 1 << 7).astype(np.int32)
    w = torch.from_numpy(w_np).cuda()
    out = None
    for _ in range(args.warmup):
        out = binding.alphabetic_tree(w)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        out = binding.alphabetic_tree(w)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(out["status"].item()) != 0:
        print(json.dumps({"error": "alphabetic tree reported an error status"}))
        return 1
    baseline = None
    if not args.no_cpu_baseline:
        baseline, (powers, _merges, M) = alphabetic_cpu_baseline(w_np)
        if int(out["cost"].item()) != M or not np.array_equal(out["powers"].cpu().numpy()[1:r], powers):
            print(json.dumps({"error": "alphabetic tree differs from the oracle"}))
            return 1
    step = wall / args.steps
    alg = 14 * r  # read the weight; write power, left, right, depth
    line = {
        "metric": ALPHA_METRIC, "value": round(r / step, 1), "unit": "leaves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"alphabetic_zipf_r{r}", "leaves": r, "weight_sum": int(w_np.sum()),
                   "weighted_path_length": int(out["cost"].item())},
        "path_roofline": {"algorithmic_bytes": alg, "frac": round(alg / step / HBM_PEAK_BPS, 5)},
        "event_ms_per_step": round(e0.elapsed_time(e1) / args.steps, 4),
        "checked_against_oracle": baseline is not None,
    }
    if baseline is not None:
        line["cpu_baseline"] = baseline
    print(json.dumps(line), flush=True)
    return 0


def alphabetic_cpu_baseline(w_np):
    """The oracle's merge order of the same weights, timed on one host core;
    returns the baseline record and the oracle's (powers, merges, M)."""
    import oracle
    t = time.perf_counter()
    res = oracle.merge_order(w_np.astype(np.int64))
    cpu_s = time.perf_counter() - t
    r = w_np.shape[0]
    return ({"value": round(r / cpu_s, 1), "unit": "leaves/s", "cores": 1, "kind": "oracle",
             "sample": f"oracle merge order of the same {r} weights, single thread on the host CPU "
                       f"({host_cpu()}), {cpu_s:.2f} s"}, res)


def run_mergecost(args) -> int:
    """Sec. 4's inputs as merge-cost experiments: for each family the GPU
    computes powersort's and peeksort's merge cost M (ps_merge_cost, keys
    untouched) and the leaf partition (ps_inspect), from which the entropy H
    of the leaf lengths follows; M/n is compared with H and H + 2 (the bounds
    of Thm. "powersort" / "peeksort").  The cpu_baseline leg runs the oracle on
    the same inputs, one pinned core: powersort (timed; its M must equal the
    GPU's) and the paper's top-down and bottom-up mergesorts with the
    already-in-order check (Sec. 4.1), whose merge costs it reports."""
    import torch
    from paper_1805_04154_amd import binding, workloads as W

    binding.load_library()
    w = args.min_run
    n24 = 1 << 24
    fams = [
        ("permutation_2p24", lambda: W.random_permutation(W.make_rng(41), n24)),
        ("random_runs_mean_sqrt_n_2p24", lambda: W.random_runs(W.make_rng(42), n24, math.sqrt(n24), 0.0)),
        ("random_runs_mean_3000_n1e7", lambda: W.random_runs(W.make_rng(0), 10 ** 7, 3000.0, 0.0)),
        ("random_runs_mean_64_2p24", lambda: W.random_runs(W.make_rng(43), n24, 64.0, 0.25)),
        ("zipf_runs_2p24", lambda: W.zipf_runs(n24, key_dtype=np.int32).keys),
    ]
    rows, host_keys = [], []
    total_keys, total_s = 0, 0.0
    for name, gen in fams:
        kn = np.ascontiguousarray(gen()).astype(np.int32)
        host_keys.append(kn)
        keys = torch.from_numpy(kn).cuda()
        n = keys.numel()
        res = {"family": name, "n": n}
        for method in ("powersort", "peeksort"):
            binding.merge_cost(keys, min_run=w, method=method)  # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                M = binding.merge_cost(keys, min_run=w, method=method)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / args.steps
            res[f"M_{method}"] = int(M.item())
            res[f"M_over_n_{method}"] = round(int(M.item()) / n, 4)
            res[f"ms_{method}"] = round(dt * 1e3, 4)
            total_keys += n
            total_s += dt
        ins = binding.inspect(keys, min_run=w)
        torch.cuda.synchronize()
        L = np.diff(ins["starts"].cpu().numpy().astype(np.int64)).astype(np.float64)
        H = float(np.sum((L / n) * np.log2(n / L)))
        res.update({"leaves": int(ins["r"]), "H": round(H, 4), "H_plus_2": round(H + 2, 4)})
        rows.append(res)
    line = {
        "metric": MERGECOST_METRIC, "value": round(total_keys / total_s, 1), "unit": "keys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(total_s * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "mergecost_families", "min_run": w}, "families": rows,
    }
    if not args.no_cpu_baseline:
        base = mergecost_cpu_baseline(fams, host_keys, rows, w)
        if "error" in base:
            print(json.dumps(base), flush=True)
            return 1
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)
    return 0


def mergecost_cpu_baseline(fams, host_keys, rows, w) -> dict:
    """The oracle on every family, one pinned core: powersort's merge cost
    (must equal the GPU's) and time, the merge costs of the paper's
    top-down and bottom-up mergesorts (Sec. 4.1), and powersort's key
    comparisons with plain and with galloping merges (Sec. 4.1, Sec. 5)."""
    import oracle

    def work():
        out, nk, secs = [], 0, 0.0
        for (name, _), k, row in zip(fams, host_keys, rows):
            n = k.shape[0]
            t = time.perf_counter()
            ps = oracle.powersort(k, None, min_run=w, details=False)
            secs += time.perf_counter() - t
            nk += n
            if ps.merge_cost != row["M_powersort"]:
                return {"error": f"{name}: the oracle's merge cost differs from the GPU's"}
            td = oracle.topdown_mergesort(k, None, min_run=w).merge_cost
            bu = oracle.bottomup_mergesort(k, None, min_run=w).merge_cost
            gal = oracle.powersort(k, None, min_run=w, details=False, galloping=True)
            if gal.merge_cost != ps.merge_cost:
                return {"error": f"{name}: galloping merges changed the oracle's merge cost"}
            out.append({"family": name, "M_over_n_powersort": round(ps.merge_cost / n, 4),
                        "M_over_n_topdown_mergesort": round(td / n, 4),
                        "M_over_n_bottomup_mergesort": round(bu / n, 4),
                        "comparisons_per_key_plain_merge": round(ps.comparisons / n, 4),
                        "comparisons_per_key_galloping_merge": round(gal.comparisons / n, 4)})
        return {"families": out, "keys": nk, "secs": secs}

    r, core = run_pinned(work)
    if "error" in r:
        return r
    return {"value": round(r["keys"] / r["secs"], 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"every family once: oracle powersort (timed), top-down and bottom-up mergesort, powersort "
                      f"with galloping merges; one "
                      f"thread pinned to host core {core} ({host_cpu()})",
            "families": r["families"]}


def sub_line(d: dict) -> dict:
    """A workload's result as a sub-object of the default line (without the
    fields every JSON line repeats)."""
    drop = {"n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"}
    return {k: v for k, v in d.items() if k not in drop}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--workload", choices=WORKLOADS, default="zipf_i32")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: print the headline alone (no latency, batched or served parts)")
    ap.add_argument("--min-run", type=int, default=24)
    ap.add_argument("--method", choices=("powersort", "peeksort"), default="powersort",
                    help="merge tree: node powers (powersort) or Alg. PeekSort's top-down tree")
    ap.add_argument("--cpu-reps", type=int, default=3, help="timed oracle calls of the headline's cpu_baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the batched and served cpu_baseline samples")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--segments", type=int, default=4096, help="arrays in the batched workload")
    ap.add_argument("--batched-reps", type=int, default=5, help="timed batched sorts (eager and graph)")
    ap.add_argument("--tune", action="store_true", help="batched: run the autotuner instead of the tuning cache")
    ap.add_argument("--duration", type=float, default=1.0, help="served: seconds of Poisson arrivals")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: arrivals per second")
    ap.add_argument("--budget-gib", type=float, default=48.0, help="served: HBM budget of the server")
    ap.add_argument("--slots", type=int, default=2, help="served: batches in flight")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration under rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the sort runs on one GPU (asked for --gpus {args.gpus}); "
              "it has no sharding or collectives", file=sys.stderr)
        return 2
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cpu = not args.no_cpu_baseline

    def emit(d: dict) -> int:
        print(json.dumps(d), flush=True)
        return 1 if "error" in d else 0

    if args.workload == "batched":
        return emit(run_batched(args, cpu))
    if args.workload == "served":
        return emit(run_served(args, cpu))
    if args.workload == "runs_2p20":
        d = run_latency(args, cpu=cpu)
        if "error" not in d:
            d.update({"n_gpus": 1, "steps": 200, "warmup": 10, "ms_per_step": d["graph_ms"]["p50"],
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                      "data": "synthetic", "config": {"workload": d.pop("workload"), "n": d["n"]}})
        return emit(d)
    if args.workload == "alphabetic":
        return run_alphabetic(args)
    if args.workload == "mergecost":
        return run_mergecost(args)

    out, wl = run_headline(args)
    if wl is None:
        return emit(out)
    if cpu:
        base = cpu_baseline(wl, args.method, args.cpu_reps)
        if base["merge_cost"] != out["config"]["merge_cost"] or not base["merge_costs_agree"]:
            return emit({"error": "the oracle's merge cost differs from the GPU's",
                         "gpu": out["config"]["merge_cost"], "oracle": base["merge_cost"]})
        out["cpu_baseline"] = base
    del wl
    composite = args.workload == "zipf_i32" and args.log2n == 28 and not args.headline_only
    if composite:
        print("bench.py: headline done; latency, batched and served parts follow", file=sys.stderr, flush=True)
        for name, fn in (("latency_2p20", run_latency), ("batched", run_batched), ("served", run_served)):
            t = time.perf_counter()
            d = fn(args, cpu=cpu)
            if "error" in d:
                return emit({"error": f"{name}: {d['error']}"})
            d["part_wall_s"] = round(time.perf_counter() - t, 1)
            out[name] = sub_line(d)
            print(f"bench.py: {name} done in {d['part_wall_s']} s", file=sys.stderr, flush=True)
    return emit(out)


if __name__ == "__main__":
    sys.exit(main())
