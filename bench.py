#!/usr/bin/env python3
"""Benchmark of the MI355X powersort on its headline workload.

One step = one ps_sort of the whole input (run detection, leaf partition,
node powers, merge tree, leaf formation and every merge) on a fresh copy of
the input that is already resident in HBM.  Default workload: n = 2^28
int32 keys with a uint32 index payload, runs of Zipf(1.2) lengths (clipped to
2^24), keys uniform in [0, 2^20), 10% strictly descending runs.

Prints one JSON line (rank 0) with keys/s, the HBM roofline of the merge-pass
kernel, the whole-path fraction of the roofline computed from the merge cost,
and the CPU oracle timed on the host as a reported baseline.

Three more regions of the same sorts are reported for information: with no
events at all, with every kernel group timed, and with one event between
consecutive sorts (median, p10 and p90 of the per-sort time).

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E
METRIC = "keys/s and % HBM roofline (2^28 int32+idx); batched/served vs plain; p50/p99"
WORKLOADS = ("zipf_i32", "zipf_u64", "perm_i32", "runs_i32", "batched", "served", "alphabetic", "mergecost")
MERGECOST_METRIC = ("merge cost M/n of powersort and peeksort (GPU ps_merge_cost) against the entropy bound and "
                    "non-adaptive mergesort, per input family; merge-cost keys/s")
ALPHA_METRIC = "alphabetic tree (Method 2') leaves/s: node powers, tree, depths and weighted path length"
SERVED_METRIC = ("served sorts: p50/p99 latency and keys/s, continuous batching vs plain per-request calls "
                 "(Poisson 2000 req/s, sizes 2^12..2^24, int32/int64/float32 keys + uint32 payload)")
BATCHED_METRIC = "batched segmented sort keys/s vs plain per-array calls (4096 arrays, log-uniform sizes 2^10..2^22)"


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


def merge_kernel_digest() -> str:
    """Digest of the merge-pass kernel's source text (its LDS struct and body)."""
    src = open(os.path.join(ROOT, "paper_1805_04154_amd", "csrc", "merge.hip")).read()
    a = src.index("template <int KT, int TILE>\nstruct MergeShared")
    a2 = src.index("\n};\n", a)
    b = src.index("template <int KT, bool HP, int NT, int IT>\n__global__ __launch_bounds__(NT) void merge_pass_kernel")
    b2 = src.index("\n}\n", b)
    return hashlib.sha256((src[a:a2] + src[b:b2]).encode()).hexdigest()[:16]


def measured_traffic(workload: str, launches_per_sort: int, merge_tile: int):
    """HBM bytes per merge-pass launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a device copy), if
    it was taken on this workload, on the current kernel source, with the
    same merge tile and number of merge launches per sort; else None."""
    try:
        text = open(COUNTERS_MD).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
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


def cpu_baseline(wl, budget_s: float, method: str = "powersort") -> dict:
    """The oracle as it stands, single-threaded on a host core, on a prefix
    of the workload sized to take roughly budget_s seconds."""
    import oracle
    sort = oracle.powersort if method == "powersort" else oracle.peeksort
    n = wl.n
    m = min(n, 1 << 22)
    t = time.perf_counter()
    sort(wl.keys[:m], wl.payload[:m], details=False)
    dt = time.perf_counter() - t
    # grow the sample while the projected time fits the budget
    while m < n and dt * 2.2 < budget_s:
        m = min(n, 2 * m)
        t = time.perf_counter()
        sort(wl.keys[:m], wl.payload[:m], details=False)
        dt = time.perf_counter() - t
    return {"value": m / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} of the {n} keys of the same workload (payload = index), one {method} call, "
                      f"single thread on the host CPU ({host_cpu()}, {os.cpu_count()} logical cores visible), "
                      f"{dt:.2f} s"}


def host_cores() -> int:
    """Cores this process may run on, at most 16 (one GPU's share of a box)."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def batched_cpu_baseline(wl, budget_s: float) -> dict:
    """The oracle on the batch's segments, each an independent powersort: one
    core in segment order for budget_s / 2, then every usable core (one
    thread each; the C oracle runs without the GIL) on the following segments
    for as long.  Segment sizes are i.i.d., so either prefix is a fair sample."""
    import threading
    import oracle
    offs = wl.offsets.astype(np.int64)
    nseg = offs.shape[0] - 1

    def one(i):
        a, b = int(offs[i]), int(offs[i + 1])
        oracle.powersort(wl.keys[a:b], wl.payload[a:b], details=False)
        return b - a

    t0 = time.perf_counter()
    k1, i = 0, 0
    while i < nseg and time.perf_counter() - t0 < budget_s / 2:
        k1 += one(i)
        i += 1
    dt1 = time.perf_counter() - t0
    first_all = i
    cores = host_cores()
    lock = threading.Lock()
    state = {"next": i, "keys": 0}
    t0 = time.perf_counter()

    def worker():
        while True:
            with lock:
                if state["next"] >= nseg or time.perf_counter() - t0 >= budget_s / 2:
                    return
                j = state["next"]
                state["next"] += 1
            kk = one(j)
            with lock:
                state["keys"] += kk

    threads = [threading.Thread(target=worker) for _ in range(cores)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dt_all = time.perf_counter() - t0
    return {"value": round(k1 / dt1, 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"segments 0..{first_all - 1} of {nseg} ({k1} keys), one oracle powersort per segment, "
                      f"single thread on the host CPU ({host_cpu()}), {dt1:.2f} s",
            "all_cores": {"value": round(state["keys"] / dt_all, 1), "unit": "keys/s", "cores": cores,
                          "sample": f"segments {first_all}..{state['next'] - 1} ({state['keys']} keys), "
                                    f"{cores} threads each running oracle calls on whole segments, {dt_all:.2f} s"}}


def served_cpu_baseline(keys_list, budget_s: float) -> dict:
    """Single-core oracle service time per request, over the trace's first
    requests until budget_s: p50/p99 of one oracle powersort call each."""
    import oracle
    from paper_1805_04154_amd import workloads as W
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
    a = np.asarray(ts) * 1e3
    return {"value": round(float(nk / (a.sum() / 1e3)), 1), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "service_ms": {"p50": round(float(np.percentile(a, 50)), 3), "p99": round(float(np.percentile(a, 99)), 3)},
            "sample": f"first {len(ts)} requests of the trace ({nk} keys), one oracle powersort call each, "
                      f"single thread on the host CPU ({host_cpu()})"}


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


def percentiles_ms(samples_s) -> dict:
    """Median, p10 and p90 of per-sort durations, in ms."""
    a = np.sort(np.asarray(samples_s, dtype=np.float64)) * 1e3
    return {"median": round(float(np.median(a)), 4), "p10": round(float(np.percentile(a, 10)), 4),
            "p90": round(float(np.percentile(a, 90)), 4), "sorts": int(a.size)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--workload", choices=WORKLOADS, default="zipf_i32")
    ap.add_argument("--min-run", type=int, default=24)
    ap.add_argument("--method", choices=("powersort", "peeksort"), default="powersort",
                    help="merge tree: node powers (powersort) or Alg. PeekSort's top-down tree")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--segments", type=int, default=4096, help="arrays in the batched workload")
    ap.add_argument("--no-tune", action="store_true", help="batched: skip the autotuner")
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
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "served":
        return run_served(args)
    if args.workload == "alphabetic":
        return run_alphabetic(args)
    if args.workload == "mergecost":
        return run_mergecost(args)

    import torch
    from paper_1805_04154_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.load_library()
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
    if not (sorted_ok and perm_ok and keys_ok and stable_ok):
        print(json.dumps({"error": "output is not the stable sort", "sorted": sorted_ok, "perm": perm_ok,
                          "keys": keys_ok, "stable": stable_ok}))
        return 1

    if args.calib_copy_mib:
        a = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

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
    traffic = (measured_traffic(wl.name, launches_per_sort, merge_tile)
               if (args.min_run == 24 and args.method == "powersort") else None)
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": peak_gbs, "unit": "GB/s",
                "frac": round(achieved_gbs / peak_gbs, 4), "traffic": traffic,
                "kernel": "merge_pass_kernel" if kb == 4 else "merge_pass_cr_kernel",
                "merge_tile": merge_tile, "launch_ms": round(mp_launch_ms, 4),
                "algorithmic_bytes_per_launch": int(mp_bytes_per_launch)}
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget, args.method)
    print(json.dumps(out), flush=True)
    return 0


def run_batched(args) -> int:
    """4096 arrays of log-uniform sizes: plain per-array ps_sort calls vs one
    ps_segmented_sort (eager and replayed as a captured hipGraph, with the
    autotuned launch shape).  Every timed sort starts from the same unsorted
    input, restored outside the timed region."""
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
        return sorted(ts)[len(ts) // 2]

    def plain():
        for g in range(nseg):
            a, c = int(offs[g]), int(offs[g + 1])
            binding.sort(b.keys[a:c], b.payload[a:c], min_run=args.min_run)

    reps = max(1, args.steps)
    plain()  # warm-up (grows the per-stream pool to the largest array)
    torch.cuda.synchronize()
    plain_ms = timed(plain, min(reps, 3))
    b.sort()
    torch.cuda.synchronize()
    eager_ms = timed(b.sort, reps)
    tuned = None
    key = autotune.signature(n, nseg, torch.int32, args.min_run, "batched_")
    if not args.no_tune:
        tuned, results = autotune.tune(restore, b.sort, autotune.candidates(), reps=2)
        autotune.save_cache(key, tuned, results[0][0])
    restore()
    b.capture()
    graph_ms = timed(b.replay, reps)
    # correctness of the last replay: per segment sorted, stable, a permutation
    restore()
    b.replay()
    torch.cuda.synchronize()
    kh = b.keys.cpu().numpy()
    ph = b.payload.view(torch.int32).cpu().numpy().view(np.uint32)
    seg_of = np.repeat(np.arange(nseg), np.diff(offs))
    ok = bool(np.array_equal(seg_of[ph], seg_of)) and bool(np.array_equal(kh, wl.keys[ph]))
    same = (seg_of[1:] == seg_of[:-1])
    ok = ok and bool(np.all(kh[1:][same] >= kh[:-1][same]))
    eq = same & (kh[1:] == kh[:-1])
    ok = ok and bool(np.all(ph[1:][eq] > ph[:-1][eq]))
    if not ok:
        print(json.dumps({"error": "batched output is not the per-segment stable sort"}))
        return 1
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
    out = {
        "metric": BATCHED_METRIC,
        "value": round(n / (graph_ms / 1e3), 1),
        "unit": "keys/s",
        "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(graph_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "segments": nseg, "key": "int32", "payload": "uint32 index",
                   "min_run": args.min_run, "merge_cost": M, "tuning": binding.get_tuning()},
        "plain": {"ms": round(plain_ms, 3), "keys_per_s": round(n / (plain_ms / 1e3), 1),
                  "calls": nseg},
        "batched_eager": {"ms": round(eager_ms, 3), "keys_per_s": round(n / (eager_ms / 1e3), 1)},
        "batched_graph": {"ms": round(graph_ms, 3), "keys_per_s": round(n / (graph_ms / 1e3), 1)},
        "speedup_vs_plain": round(plain_ms / best_ms, 2),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_BPS / 1e9, "unit": "GB/s",
                     "frac": round(ach / (HBM_PEAK_BPS / 1e9), 4), "traffic": None, "kernel": "merge_pass_kernel",
                     "launch_ms": round(mp_ms, 4)},
        "path_roofline": {"algorithmic_bytes": b_alg, "frac": round(b_alg / (best_ms / 1e3) / HBM_PEAK_BPS, 4)},
        "kernel_groups_ms": groups,
        "gen_s": round(t_gen, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batched_cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


def run_served(args) -> int:
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
        out_runs[f"batched_{name}"] = serving.latency_stats(done)
        if name == "saturated":
            # results of the saturated batched run: per-request stable sort
            for r in done[:: max(1, len(done) // 16)]:
                kh = r.keys.cpu().numpy().view(keys[r.rid].dtype)
                ph = r.payload.view(torch.int32).cpu().numpy().view(np.uint32)
                if not np.array_equal(kh.view(np.uint8), keys[r.rid][ph].view(np.uint8)):
                    print(json.dumps({"error": "served output is not a permutation of the request"}))
                    return 1
        reqs = fresh()
        done = serving.serve_plain(reqs, min_run=args.min_run, realtime=realtime)
        out_runs[f"plain_{name}"] = serving.latency_stats(done)
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = served_cpu_baseline(keys, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


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


def topdown_merge_cost(n: int, w: int) -> int:
    """Merge cost of non-adaptive top-down mergesort that insertion-sorts
    subarrays of at most w elements: n + M(floor(n/2)) + M(ceil(n/2))."""
    memo = {}

    def m(k):
        if k <= w:
            return 0
        if k not in memo:
            memo[k] = k + m(k // 2) + m(k - k // 2)
        return memo[k]
    return m(n)


def bottomup_merge_cost(n: int, w: int) -> int:
    """Merge cost of non-adaptive bottom-up mergesort over blocks of w
    elements, merging neighbours level by level (an odd block passes up)."""
    runs = [w] * (n // w) + ([n % w] if n % w else [])
    M = 0
    while len(runs) > 1:
        nxt = []
        for i in range(0, len(runs) - 1, 2):
            nxt.append(runs[i] + runs[i + 1])
            M += runs[i] + runs[i + 1]
        if len(runs) % 2:
            nxt.append(runs[-1])
        runs = nxt
    return M


def run_mergecost(args) -> int:
    """Sec. 4's inputs as merge-cost experiments: for each family the GPU
    computes powersort's and peeksort's merge cost M (ps_merge_cost, keys
    untouched) and the leaf partition (ps_inspect), from which the entropy H
    of the leaf lengths follows; M/n is compared with H, H + 2 (the bounds of
    Thm. "powersort" / "peeksort") and with non-adaptive mergesort."""
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
    rows = []
    total_keys, total_s = 0, 0.0
    for name, gen in fams:
        keys = torch.from_numpy(np.ascontiguousarray(gen()).astype(np.int32)).cuda()
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
            res[f"M_over_n_{method}"] = round(int(M.item()) / n, 4)
            res[f"ms_{method}"] = round(dt * 1e3, 4)
            total_keys += n
            total_s += dt
        ins = binding.inspect(keys, min_run=w)
        torch.cuda.synchronize()
        L = np.diff(ins["starts"].cpu().numpy().astype(np.int64)).astype(np.float64)
        H = float(np.sum((L / n) * np.log2(n / L)))
        res.update({"leaves": int(ins["r"]), "H": round(H, 4), "H_plus_2": round(H + 2, 4),
                    "topdown_mergesort": round(topdown_merge_cost(n, w) / n, 4),
                    "bottomup_mergesort": round(bottomup_merge_cost(n, w) / n, 4)})
        rows.append(res)
    print(json.dumps({
        "metric": MERGECOST_METRIC, "value": round(total_keys / total_s, 1), "unit": "keys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(total_s * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "mergecost_families", "min_run": w}, "families": rows,
    }), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
