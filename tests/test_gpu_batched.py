"""Batched sorting through ps_segmented_sort: eager, replayed as a captured
hipGraph, and under every tuned launch shape, always equal to the oracle."""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import batched, binding
    binding.load_library()
    binding.set_tuning(None)
    wl = W.batched_random_runs(nseg=300, lo_exp=4, hi_exp=15, workers=1)
    import oracle
    rk, rp, rc = oracle.segmented_powersort(wl.keys, wl.payload, wl.offsets)
    return batched, binding, wl, (rk, rp, rc)


def run_eager(batched, wl):
    import torch
    b = batched.SegmentedBatch(wl.offsets, wl.keys.dtype)
    b.load(to_dev(wl.keys), to_dev(wl.payload))
    b.sort()
    torch.cuda.synchronize()
    return b


def test_eager_matches_oracle(setup):
    batched, binding, wl, (rk, rp, rc) = setup
    b = run_eager(batched, wl)
    assert int(b.status.item()) == 0
    assert np.array_equal(to_host(b.keys, np.int32), rk)
    assert np.array_equal(to_host(b.payload, np.uint32), rp)
    assert np.array_equal(b.costs.cpu().numpy().view(np.uint64), rc)


def test_graph_replays_match_eager(setup):
    import torch
    batched, binding, wl, (rk, rp, rc) = setup
    b = batched.SegmentedBatch(wl.offsets, wl.keys.dtype)
    src_k, src_p = to_dev(wl.keys), to_dev(wl.payload)
    b.load(src_k, src_p)
    b.capture()  # eager warm-up + capture
    other = to_dev(W.random_permutation(W.make_rng(77), 50000).astype(np.int32))
    for rep in range(4):
        b.load(src_k, src_p)  # eager work between replays
        torch.cuda.synchronize()
        b.costs.zero_()
        b.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(b.keys, np.int32), rk), f"replay {rep}"
        assert np.array_equal(to_host(b.payload, np.uint32), rp), f"replay {rep}"
        assert np.array_equal(b.costs.cpu().numpy().view(np.uint64), rc), f"replay {rep}"
        # an unrelated eager sort on the same stream between replays
        o = other.clone()
        binding.sort(o)
        torch.cuda.synchronize()
        assert bool((o[1:] >= o[:-1]).all())


def test_tunings_do_not_change_results(setup):
    import torch
    batched, binding, wl, (rk, rp, rc) = setup
    try:
        for t in ({"merge_tile": 2048}, {"merge_tile": 4096, "grid_merge": 64, "grid_split": 3},
                  {"merge_tile": 2048, "grid_fused": 5, "grid_big_leaf": 7, "grid_merge": 4096},
                  {"merge_tile": 8192}, {"merge_tile": 8192, "grid_merge": 37, "grid_split": 5}):
            binding.set_tuning(t)
            b = run_eager(batched, wl)
            assert np.array_equal(to_host(b.keys, np.int32), rk), t
            assert np.array_equal(to_host(b.payload, np.uint32), rp), t
            assert np.array_equal(b.costs.cpu().numpy().view(np.uint64), rc), t
    finally:
        binding.set_tuning(None)


def test_autotuner_picks_a_candidate_and_keeps_results(setup, tmp_path):
    import torch
    from paper_1805_04154_amd import autotune
    batched, binding, wl, (rk, rp, rc) = setup
    b = batched.SegmentedBatch(wl.offsets, wl.keys.dtype)
    src_k, src_p = to_dev(wl.keys), to_dev(wl.payload)
    cands = autotune.candidates(small=True)
    try:
        best, results = autotune.tune(lambda: b.load(src_k, src_p), b.sort, cands, reps=2)
        assert best in cands and len(results) == len(cands)
        key = autotune.signature(b.n, b.nseg, torch.int32, None, "test_")
        path = str(tmp_path / "tuning.json")
        autotune.save_cache(key, best, results[0][0], path)
        binding.set_tuning(None)
        assert autotune.apply_cached(key, path) == best
        b.load(src_k, src_p)
        b.sort()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(b.keys, np.int32), rk)
        assert np.array_equal(to_host(b.payload, np.uint32), rp)
    finally:
        binding.set_tuning(None)


def test_single_sort_graph_replays_match_eager(setup):
    """One ps_sort with a caller workspace captured as a graph (as the
    single-sort latency benchmark does) and replayed four times, with eager
    work and synchronisations between replays: every replay equals the
    oracle."""
    import torch
    import oracle
    batched, binding, wl, _ = setup
    one = W.runs_2p20(n=(1 << 20) + 3)
    ref = oracle.powersort(one.keys, one.payload, details=False)
    src_k, src_p = to_dev(one.keys), to_dev(one.payload)
    k, p = src_k.clone(), src_p.clone()
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(binding.workspace_bytes(one.n, 1, torch.int32, True), dtype=torch.uint8, device="cuda")
    binding.sort(k, p, merge_cost=M, workspace=ws)  # eager warm-up
    torch.cuda.synchronize()
    k.copy_(src_k)
    p.copy_(src_p)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        binding.sort(k, p, merge_cost=M, workspace=ws)
    torch.cuda.synchronize()
    other = to_dev(W.random_permutation(W.make_rng(78), 30000).astype(np.int32))
    for rep in range(4):
        k.copy_(src_k)
        p.copy_(src_p)
        M.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(k, np.int32), ref.keys), f"replay {rep}"
        assert np.array_equal(to_host(p, np.uint32), ref.payload), f"replay {rep}"
        assert int(M.item()) == ref.merge_cost, f"replay {rep}"
        o = other.clone()
        binding.sort(o)  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert bool((o[1:] >= o[:-1]).all())
