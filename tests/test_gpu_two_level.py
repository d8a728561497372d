"""Two-level merge passes (ps_tuning.merge_levels = 2): a big node at odd
depth is merged in the same pass as its parent, which then merges up to four
inputs.  Every result must still be the oracle's stable sort and merge cost:
long leaves at every depth with three and two data arrays, peeksort's tree,
segmented batches, every key type and minimum run, the merge tiles, and the
benchmark inputs at full size.  The merge group's element count shows that
nodes were absorbed."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host
from tests.test_gpu_parity import cast_keys
from tests.test_gpu_placement import long_leaf_input, placement_inputs, run_sort

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    binding.set_tuning({"merge_levels": 2})
    yield binding
    binding.set_tuning(None)


def merged_elements(ps, keys_np, levels):
    """Elements written by the merge passes of one sort at merge_levels."""
    import torch
    ps.set_tuning({"merge_levels": levels})
    ps.profile_enable(True)
    ps.profile_read(reset=True)
    k = to_dev(keys_np)
    ps.sort(k)
    torch.cuda.synchronize()
    pr = ps.profile_read(reset=True)
    ps.profile_enable(False)
    ps.set_tuning({"merge_levels": 2})
    return pr["merge"]["elems"]


def test_nodes_are_absorbed(ps):
    keys = W.runs_sqrt_i32(1 << 22).keys
    one, two = merged_elements(ps, keys, 1), merged_elements(ps, keys, 2)
    assert 0 < two < 0.8 * one


@pytest.mark.parametrize("compact", [False, True])
@pytest.mark.parametrize("dtype,with_payload", [(np.int32, True), (np.int32, False), (np.float32, True),
                                                (np.uint64, True)])
def test_long_leaves_at_every_depth(ps, compact, dtype, with_payload):
    import oracle
    for seed, v in placement_inputs():
        keys = cast_keys(v, dtype)
        ref = oracle.powersort(keys, np.arange(keys.shape[0], dtype=np.uint32) if with_payload else None)
        gk, gp, gm = run_sort(ps, keys, with_payload, compact)
        assert np.array_equal(gk.view(np.uint8), ref.keys.view(np.uint8)), seed
        if with_payload:
            assert np.array_equal(gp, ref.payload), seed
        assert gm == ref.merge_cost, seed


@pytest.mark.parametrize("compact", [False, True])
def test_peeksort(ps, compact):
    import oracle
    for seed in range(60, 66):
        keys = long_leaf_input(seed).astype(np.int32)
        ref = oracle.peeksort(keys, np.arange(keys.shape[0], dtype=np.uint32))
        gk, gp, gm = run_sort(ps, keys, True, compact, method="peeksort")
        assert np.array_equal(gk, ref.keys) and np.array_equal(gp, ref.payload) and gm == ref.merge_cost, seed
    wl = W.runs_sqrt_i32(1 << 21)
    ref = oracle.peeksort(wl.keys, wl.payload)
    gk, gp, gm = run_sort(ps, wl.keys, True, compact, method="peeksort")
    assert np.array_equal(gk, ref.keys) and np.array_equal(gp, ref.payload) and gm == ref.merge_cost


@pytest.mark.parametrize("compact", [False, True])
def test_segmented(ps, compact):
    import torch
    import oracle
    parts = [long_leaf_input(70 + g) for g in range(5)] + [np.arange(9000)[::-1].copy(), np.zeros(0, np.int64)]
    parts += [W.random_runs(W.make_rng(90 + g), 200_000 + 7 * g, 300.0, 0.25) for g in range(4)]
    offsets = np.zeros(len(parts) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(p) for p in parts])
    keys = np.concatenate(parts).astype(np.int32)
    pay = np.arange(len(keys), dtype=np.uint32)
    rk, rp, rc = oracle.segmented_powersort(keys, pay, offsets)
    k, p = to_dev(keys), to_dev(pay)
    off = torch.from_numpy(offsets.view(np.int64)).cuda()
    costs = torch.zeros(len(parts), dtype=torch.int64, device="cuda")
    ps.segmented_sort(k, p, off, merge_costs=costs, compact_scratch=compact)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(k, np.int32), rk)
    assert np.array_equal(to_host(p, np.uint32), rp)
    assert np.array_equal(costs.cpu().numpy().view(np.uint64), rc)


@pytest.mark.parametrize("w", [1, 2, 24, 64])
@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.float32, np.int64])
def test_inputs_and_min_runs(ps, w, dtype):
    import oracle
    rng = W.make_rng(400 + w)
    for n in (0, 1, 2, 4097, 70_001, 600_000):
        for v in (W.random_permutation(rng, n), W.random_runs(rng, n, max(2.0, n ** 0.5), 0.25),
                  rng.integers(0, 7, size=n)):
            keys = cast_keys(np.asarray(v, dtype=np.int64), dtype)
            pay = np.arange(n, dtype=np.uint32)
            ref = oracle.powersort(keys, pay, min_run=w)
            k, p = to_dev(keys), to_dev(pay)
            import torch
            M = torch.zeros(1, dtype=torch.int64, device="cuda")
            ps.sort(k, p, min_run=w, merge_cost=M)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(k, keys.dtype).view(np.uint8), ref.keys.view(np.uint8)), (n, w)
            assert np.array_equal(to_host(p, np.uint32), ref.payload), (n, w)
            assert int(M.item()) == ref.merge_cost, (n, w)


@pytest.mark.parametrize("tile", [2048, 4096, 8192])
def test_merge_tiles(ps, tile):
    import oracle
    wl = W.runs_sqrt_i32(1 << 22)
    ref = oracle.powersort(wl.keys, wl.payload)
    try:
        ps.set_tuning({"merge_tile": tile, "merge_levels": 2, "grid_merge": 333, "grid_split": 77})
        gk, gp, gm = run_sort(ps, wl.keys, True, False)
    finally:
        ps.set_tuning({"merge_levels": 2, "merge_tile": 8192, "grid_merge": 2048, "grid_split": 2048})
    assert np.array_equal(gk, ref.keys) and np.array_equal(gp, ref.payload) and gm == ref.merge_cost


@pytest.mark.parametrize("name", ["zipf_i32_2p28", "perm_i32_2p26", "runs_i32_2p26"])
def test_benchmark_inputs_full_size(ps, name):
    import torch
    import oracle
    print(f"two-level passes, full size: {name}", flush=True)
    wl = {"zipf_i32_2p28": lambda: W.zipf_runs(1 << 28, key_dtype=np.int32),
          "perm_i32_2p26": lambda: W.permutation_i32(1 << 26),
          "runs_i32_2p26": lambda: W.runs_sqrt_i32(1 << 26)}[name]()
    ref = oracle.powersort(wl.keys, wl.payload, details=False)
    gk, gp, gm = run_sort(ps, wl.keys, True, False)
    assert gm == ref.merge_cost
    assert np.array_equal(gp, ref.payload)
    assert np.array_equal(gk, ref.keys)
    torch.cuda.empty_cache()
