"""Where long leaves are merged from.  With three data arrays (the default) a
leaf longer than a fused subtree (4096 elements) stays in the caller's array,
reversed there if it is decreasing, unless its parent is the root; with
PS_FLAG_COMPACT_SCRATCH (two arrays) it is copied to scratch when its depth
is odd.  Both must produce the oracle's stable sort and merge cost.  The
inputs put long ascending and strictly descending leaves at depths 0 to 4 and
deeper, beside short leaves, fused subtrees and long merges; the test checks
that coverage through ps_inspect's leaf depths."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host
from tests.test_gpu_parity import cast_keys

pytestmark = pytest.mark.gpu

KFUSE = 4096


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    return binding


def long_leaf_input(seed: int) -> np.ndarray:
    """Long runs (4097..30000 elements, half of them strictly descending) separated by
    short random-run stretches (0..3000 elements).  Every third seed adds, in
    front or at the back, one run longer than all the rest together, which
    makes it a child of the root."""
    rng = W.make_rng(seed)
    parts = []
    for _ in range(int(rng.integers(3, 14))):
        base = rng.integers(0, 1 << 20, size=int(rng.integers(4097, 30000)))
        if rng.random() < 0.5:
            run = np.unique(base)[::-1]  # strictly descending (a few values collide and drop)
        else:
            run = np.sort(base)
        parts.append(run)
        m = int(rng.integers(0, 3000))
        if m:
            parts.append((W.random_runs(rng, m, 20.0, 0.25) * 37) % (1 << 20))
    if seed % 3 == 0:
        total = sum(len(p) for p in parts)
        big = np.arange(total + 5000, dtype=np.int64) * 3
        if seed % 2:
            big = big[::-1]
        parts = [big] + parts if seed % 4 else parts + [big]
    return np.concatenate(parts).astype(np.int64)


def three_runs(dirs, sizes) -> np.ndarray:
    """Three natural runs of the given sizes and directions (True =
    strictly descending), each boundary a break.  With sizes (a, a, 2a) the
    root merges the first two runs' node with the third run, so the first two
    sit at depth 2 and the third at depth 1; (2a, a, a) mirrors that."""
    parts, first = [], 10_000_000
    for size, desc in zip(sizes, dirs):
        run = first - 2 * np.arange(size) if desc else first + 2 * np.arange(size)
        parts.append(run)
        # an ascending run breaks at a smaller value, a descending one at a larger
        first = int(run[-1]) + (1 if desc else -1)
    return np.concatenate(parts).astype(np.int64)


def placement_inputs():
    for seed in range(40, 52):
        yield f"seed{seed}", long_leaf_input(seed)
    for sizes in ((10000, 10000, 20000), (20000, 10000, 10000)):
        for m in range(8):
            dirs = (bool(m & 1), bool(m & 2), bool(m & 4))
            yield f"three{sizes}{dirs}", three_runs(dirs, sizes)


def run_sort(ps, keys_np, with_payload, compact, method="powersort"):
    import torch
    k = to_dev(keys_np)
    p = to_dev(np.arange(keys_np.shape[0], dtype=np.uint32)) if with_payload else None
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ps.sort(k, p, merge_cost=M, method=method, compact_scratch=compact)
    torch.cuda.synchronize()
    return to_host(k, keys_np.dtype), (to_host(p, np.uint32) if with_payload else None), int(M.item())


def long_leaf_depths(ps, keys_np):
    """(depth, descending) of every leaf longer than KFUSE, from ps_inspect."""
    import torch
    got = ps.inspect(to_dev(keys_np))
    torch.cuda.synchronize()
    starts = got["starts"].cpu().numpy().astype(np.int64)
    depth = got["leaf_depth"].cpu().numpy().astype(np.int64)
    out = []
    for i in range(got["r"]):
        s, e = starts[i], starts[i + 1]
        if e - s > KFUSE:
            out.append((int(depth[i]), bool(keys_np[s + 1] < keys_np[s])))
    return out


@pytest.mark.parametrize("compact", [False, True])
@pytest.mark.parametrize("dtype,with_payload", [(np.int32, True), (np.int32, False), (np.uint64, True),
                                                (np.float32, True)])
def test_long_leaves_at_every_depth(ps, compact, dtype, with_payload):
    import oracle
    seen = set()
    for seed, v in placement_inputs():
        keys = cast_keys(v, dtype)
        ref = oracle.powersort(keys, np.arange(keys.shape[0], dtype=np.uint32) if with_payload else None)
        gk, gp, gm = run_sort(ps, keys, with_payload, compact)
        assert np.array_equal(gk.view(np.uint8), ref.keys.view(np.uint8)), seed
        if with_payload:
            assert np.array_equal(gp, ref.payload), seed
        assert gm == ref.merge_cost, seed
        seen.update((min(d, 4), desc) for d, desc in long_leaf_depths(ps, keys))
    # long leaves, both directions, at depth 1 (child of the root), at even
    # and odd depths below it
    for d in (1, 2, 3):
        assert (d, False) in seen and (d, True) in seen, sorted(seen)


@pytest.mark.parametrize("compact", [False, True])
def test_whole_input_one_long_leaf(ps, compact):
    # the root is a leaf: nothing to merge, a descending run reversed in place
    for keys in (np.arange(50000, dtype=np.int32), np.arange(50000, dtype=np.int32)[::-1].copy()):
        gk, gp, gm = run_sort(ps, keys, True, compact)
        assert np.array_equal(gk, np.arange(50000, dtype=np.int32))
        assert np.array_equal(gp, np.arange(50000, dtype=np.uint32) if keys[0] == 0
                              else np.arange(50000, dtype=np.uint32)[::-1])
        assert gm == 0


@pytest.mark.parametrize("compact", [False, True])
def test_peeksort_long_leaves(ps, compact):
    import oracle
    for seed in range(60, 66):
        keys = long_leaf_input(seed).astype(np.int32)
        ref = oracle.peeksort(keys, np.arange(keys.shape[0], dtype=np.uint32))
        gk, gp, gm = run_sort(ps, keys, True, compact, method="peeksort")
        assert np.array_equal(gk, ref.keys) and np.array_equal(gp, ref.payload) and gm == ref.merge_cost, seed


@pytest.mark.parametrize("compact", [False, True])
def test_segmented_long_leaves(ps, compact):
    import torch
    import oracle
    parts = [long_leaf_input(70 + g) for g in range(5)] + [np.arange(9000)[::-1].copy(), np.zeros(0, np.int64)]
    sizes = [len(p) for p in parts]
    offsets = np.zeros(len(parts) + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
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
