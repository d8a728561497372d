"""Parity of the HIP powersort (through the C ABI) with the CPU oracle.

Bit-exact: sorted keys, payload order, merge cost M, and the intermediate
results of the method (leaf starts, node powers, the merge tree as a set of
(lo, mid, hi) merges, leaf depths)."""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import merges_from_ranges, oracle_leaf_depths, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    return binding


def small_inputs(seed):
    rng = W.make_rng(seed)
    sizes = [0, 1, 2, 3, 5, 23, 24, 25, 48, 100, 1000, 4095, 4096, 4097, 8191, 12289, 70001]
    for n in sizes:
        yield f"alpha3_{n}", rng.integers(0, 3, size=n)
        yield f"runs_{n}", W.random_runs(rng, n, max(2.0, math.sqrt(n)), 0.25) if n else np.zeros(0, np.int64)
        yield f"perm_{n}", W.random_permutation(rng, n)
    for n in (5000, 20000, 100000):
        yield f"sorted_{n}", np.arange(n)
        yield f"reversed_{n}", np.arange(n)[::-1].copy()
        yield f"equal_{n}", np.full(n, 7)
        yield f"sawtooth_{n}", np.arange(n) % 97
        yield f"longruns_{n}", W.concatenated_runs(rng, n, lambda r, k: r.integers(1, 20000, size=k), 0, 1 << 30, 0.3)


def cast_keys(v: np.ndarray, dtype):
    if dtype == np.float32:
        return (v - (v.max() // 2 if v.size else 0)).astype(np.float32)
    if dtype == np.uint64:
        return v.astype(np.uint64) * np.uint64(1 << 33) + np.uint64(5)
    if dtype == np.int64:
        return (v.astype(np.int64) - 1000) * np.int64(1 << 31)
    if dtype == np.int32:
        return (v - 50).astype(np.int32)
    return v.astype(dtype)


def check_sort(ps, keys_np, w, with_payload=True):
    import torch
    n = keys_np.shape[0]
    pay_np = np.arange(n, dtype=np.uint32)
    ref = oracle_sort(keys_np, pay_np if with_payload else None, w)
    k = to_dev(keys_np)
    p = to_dev(pay_np) if with_payload else None
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ps.sort(k, p, min_run=w, merge_cost=M)
    torch.cuda.synchronize()
    got_k = to_host(k, keys_np.dtype)
    assert np.array_equal(got_k.view(np.uint8), ref.keys.view(np.uint8)), "keys differ"
    if with_payload:
        assert np.array_equal(to_host(p, np.uint32), ref.payload), "payload order differs"
    assert int(M.item()) == ref.merge_cost, (int(M.item()), ref.merge_cost)
    return ref


def oracle_sort(keys, pay, w):
    import oracle
    return oracle.powersort(keys, pay, min_run=w)


@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.int64, np.uint64, np.float32])
@pytest.mark.parametrize("w", [1, 24])
def test_small_inputs_sort_and_cost(ps, dtype, w):
    for name, v in small_inputs(1):
        keys = cast_keys(np.asarray(v), dtype)
        try:
            check_sort(ps, keys, w)
        except AssertionError as e:
            raise AssertionError(f"case {name} dtype {np.dtype(dtype).name} w {w}: {e}")


@pytest.mark.parametrize("w", [2, 3, 7, 64])
def test_other_min_runs(ps, w):
    for name, v in small_inputs(2):
        if len(v) > 20000:
            continue
        try:
            check_sort(ps, cast_keys(np.asarray(v), np.int32), w)
        except AssertionError as e:
            raise AssertionError(f"case {name} w {w}: {e}")


def test_without_payload(ps):
    for name, v in small_inputs(3):
        check_sort(ps, cast_keys(np.asarray(v), np.int32), 24, with_payload=False)


@pytest.mark.parametrize("w", [1, 24])
def test_intermediates_match_oracle(ps, w):
    import torch
    for name, v in small_inputs(4):
        keys = cast_keys(np.asarray(v), np.int32)
        n = len(keys)
        if n == 0:
            continue
        ref = oracle_sort(keys, None, w)
        got = ps.inspect(to_dev(keys), min_run=w)
        torch.cuda.synchronize()
        assert got["r"] == ref.r, name
        starts = got["starts"].cpu().numpy().astype(np.int64)
        assert np.array_equal(starts, ref.starts.astype(np.int64)), name
        powers = got["powers"].cpu().numpy()
        assert np.array_equal(powers[1:ref.r], ref.powers), name
        left = got["node_left"].cpu().numpy()
        right = got["node_right"].cpu().numpy()
        assert merges_from_ranges(starts, powers, left, right) == {tuple(int(x) for x in m) for m in ref.merges}, name
        depth = got["leaf_depth"].cpu().numpy().astype(np.int64)
        assert np.array_equal(depth, oracle_leaf_depths(ref.starts, ref.merges)), name


def test_merge_cost_entry_leaves_keys_untouched(ps):
    import torch
    for name, v in small_inputs(5):
        keys = cast_keys(np.asarray(v), np.int32)
        ref = oracle_sort(keys, None, 24)
        k = to_dev(keys)
        M = ps.merge_cost(k, min_run=24)
        torch.cuda.synchronize()
        assert int(M.item()) == ref.merge_cost, name
        assert np.array_equal(to_host(k, np.int32), keys), name


def test_workload_runs_2p20_full(ps):
    wl = W.runs_2p20()
    ref = check_sort(ps, wl.keys, 24)
    assert ref.r > 100


def test_float_specials(ps):
    rng = W.make_rng(9)
    vals = W.random_runs(rng, 50000, 200, 0.25)
    keys = W.f32_from_values(rng, vals, 50000)
    check_sort(ps, keys, 24)


def test_determinism(ps):
    import torch
    wl = W.runs_sqrt_i32(1 << 21)
    outs = []
    for _ in range(2):
        k, p = to_dev(wl.keys), to_dev(wl.payload)
        ps.sort(k, p)
        torch.cuda.synchronize()
        outs.append((to_host(k, np.int32), to_host(p, np.uint32)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# ------------------------------------------------------------------ segmented

def segmented_case(seed, nseg, max_size):
    rng = W.make_rng(seed)
    sizes = rng.integers(0, max_size, size=nseg)
    sizes[:3] = [0, 1, 2][:min(3, nseg)]
    offsets = np.zeros(nseg + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
    parts = [W.random_runs(rng, int(s), max(2.0, math.sqrt(s)), 0.25) if s else np.zeros(0, np.int64) for s in sizes]
    keys = np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)
    return keys, offsets


@pytest.mark.parametrize("nseg,max_size", [(1, 5000), (7, 300), (100, 9000), (400, 50)])
def test_segmented_matches_oracle(ps, nseg, max_size):
    import torch
    import oracle
    keys, offsets = segmented_case(nseg * 13 + max_size, nseg, max_size)
    pay = np.arange(len(keys), dtype=np.uint32)
    rk, rp, rc = oracle.segmented_powersort(keys, pay, offsets)
    k, p = to_dev(keys), to_dev(pay)
    off = torch.from_numpy(offsets.view(np.int64)).cuda()
    costs = torch.zeros(nseg, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    ps.segmented_sort(k, p, off, merge_costs=costs, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(to_host(k, np.int32), rk)
    assert np.array_equal(to_host(p, np.uint32), rp)
    assert np.array_equal(costs.cpu().numpy().view(np.uint64), rc)
    mc = ps.segmented_merge_cost(to_dev(keys), off)
    torch.cuda.synchronize()
    assert np.array_equal(mc.cpu().numpy().view(np.uint64), rc)


def test_segmented_bad_offsets_reported(ps):
    import torch
    keys = np.arange(100, dtype=np.int32)[::-1].copy()
    k = to_dev(keys)
    off = torch.tensor([0, 60, 40, 100], dtype=torch.int64, device="cuda")  # decreasing
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ps.segmented_sort(k, None, off, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == -1
    off = torch.tensor([0, 60, 90], dtype=torch.int64, device="cuda")  # does not end at n
    ps.segmented_sort(k, None, off, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == -1


def boundary_cases():
    """Long runs whose boundaries sit at or next to 4096-position tile edges,
    in both directions, plus runs that end exactly where a window ends."""
    T = 4096
    for edge in (T, 2 * T, 3 * T):
        for delta in (-2, -1, 0, 1, 2):
            b = edge + delta
            n = 5 * T + 77
            # strictly descending up to b (inclusive of b-1), ascending after
            left = np.arange(b, 0, -1) * 3
            right = np.arange(n - b) * 3 + 1
            yield f"desc_then_asc_{b}", np.concatenate([left, right])
            # ascending then strictly descending
            yield f"asc_then_desc_{b}", np.concatenate([np.arange(b), 10 ** 6 - np.arange(n - b)])
            # ascending, then a drop, then ascending (equal keys across the drop)
            yield f"asc_drop_asc_{b}", np.concatenate([np.arange(b) // 5, np.arange(n - b) // 5])
    for L in (T - 70, T - 65, T - 64, T + 60, T + 65):
        v = np.concatenate([np.arange(L)[::-1], np.arange(2 * T) + 10 ** 5, np.arange(T)[::-1]])
        yield f"window_edge_{L}", v


@pytest.mark.parametrize("w", [1, 2, 3, 24, 64])
def test_runs_at_tile_boundaries(ps, w):
    for name, v in boundary_cases():
        try:
            check_sort(ps, v.astype(np.int32), w)
        except AssertionError as e:
            raise AssertionError(f"case {name} w {w}: {e}")


def test_pool_limit_fails_with_nothing_enqueued():
    """With the library's pool capped below what a sort needs, the call
    raises PS_ERR_OUT_OF_MEMORY and leaves the keys untouched; without the
    cap the same call sorts."""
    import torch
    from paper_1805_04154_amd import binding
    binding.load_library()
    wl = W.runs_2p20(n=1 << 20)
    k, p = to_dev(wl.keys), to_dev(wl.payload)
    s = torch.cuda.Stream()  # a stream without a pool entry yet
    need = binding.workspace_bytes(wl.n, 1, torch.int32, True)
    try:
        binding.set_pool_limit(need - 1)
        with pytest.raises(binding.PowersortError) as e:
            binding.sort(k, p, stream=s)
        assert e.value.status == -3
    finally:
        binding.set_pool_limit(0)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(k, np.int32), wl.keys)
    assert np.array_equal(to_host(p, np.uint32), wl.payload)
    binding.sort(k, p, stream=s)
    s.synchronize()
    assert bool((k[1:] >= k[:-1]).all())
    binding.release(s)
