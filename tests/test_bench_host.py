"""Host-side logic of bench.py: the gate on the committed merge-pass counter
figure, the per-sort percentiles, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def committed_fields():
    return bench.profile_fields(bench.COUNTERS_MD)


def test_traffic_gate_matches_only_what_was_measured():
    f = committed_fields()
    wl, launches, tile = f["workload"], int(f["merge_launches_per_sort"]), int(f["merge_tile"])
    got = bench.measured_traffic(wl, launches, tile)
    if f["kernel_source_digest"] != bench.merge_kernel_digest():
        # the kernel changed since the counters were taken: no figure
        assert got is None
        return
    assert got == int(f["hbm_bytes_per_launch"])
    # no more than a few percent above the algorithmic bytes it states
    alg = int(f["algorithmic bytes per launch"].split()[0])
    assert alg <= got < 1.05 * alg
    assert bench.measured_traffic(wl + "_other", launches, tile) is None
    assert bench.measured_traffic(wl, launches + 1, tile) is None
    assert bench.measured_traffic(wl, launches, 4096 if tile != 4096 else 2048) is None


def test_percentiles_ms():
    p = bench.percentiles_ms([0.001 * i for i in range(1, 11)])  # 1..10 ms
    assert p["sorts"] == 10
    assert p["median"] == 5.5
    assert abs(p["p10"] - 1.9) < 1e-9 and abs(p["p90"] - 9.1) < 1e-9
    assert bench.percentiles_ms(np.array([0.002]))["median"] == 2.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batched_and_served_oracle_baselines():
    # bounded samples: whole segments (requests) in order, never past the input
    from paper_1805_04154_amd import workloads as W
    wl = W.batched_random_runs(nseg=8)
    r = bench.batched_cpu_baseline(wl, 1.0)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert 1 <= r["all_cores"]["cores"] <= 16 and r["all_cores"]["value"] > 0
    metas = W.trace_meta(rate_hz=2000, duration_s=0.01, lo_exp=8, hi_exp=12, seed_index=11)
    keys = W.materialize(metas, workers=1)
    s = bench.served_cpu_baseline(keys, 1.0)
    assert s["service_ms"]["p50"] <= s["service_ms"]["p99"] and s["value"] > 0


def test_trace_gate_matches_only_what_was_traced():
    f = bench.profile_fields(bench.TRACE_MD)
    if "merge_pass_average_ns" not in f:
        assert bench.traced_launch_ms("zipf_runs_n268435456_int32", 8192) is None
        return
    got = bench.traced_launch_ms(f["workload"], int(f["merge_tile"]))
    if f["kernel_source_digest"] != bench.merge_kernel_digest():
        assert got is None
        return
    assert got == float(f["merge_pass_average_ns"]) / 1e6
    assert bench.traced_launch_ms(f["workload"] + "_other", int(f["merge_tile"])) is None


def test_oracle_runs_pinned_with_warmup_and_median():
    import os
    from paper_1805_04154_amd import workloads as W
    seen = []
    _, core = bench.run_pinned(lambda: seen.append(os.sched_getaffinity(0)))
    assert seen == [{core}]
    assert os.sched_getaffinity(0) != {core} or len(bench.usable_cores()) == 1  # the caller is not pinned
    wl = W.runs_2p20(n=1 << 16)
    r = bench.cpu_baseline(wl, "powersort", reps=3)
    assert r["cores"] == 1 and r["kind"] == "oracle" and len(r["times_s"]) == 3
    assert r["merge_costs_agree"] and r["merge_cost"] > 0
    assert abs(r["median_s"] - sorted(r["times_s"])[1]) < 1e-3


def test_latency_percentiles():
    p = bench.latency_ms([0.001 * i for i in range(1, 101)])
    assert p["sorts"] == 100 and p["min"] == 1.0 and p["max"] == 100.0
    assert p["p50"] == 50.5 and abs(p["p99"] - 99.01) < 1e-9
