"""Host-side logic that needs no GPU: the seeded generators, the serving
statistics and the autotuner's search space."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W


def test_generators_are_deterministic():
    a = W.runs_2p20()
    b = W.runs_2p20()
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.payload, b.payload)
    assert np.array_equal(a.payload, np.arange(a.n, dtype=np.uint32))
    z1 = W.zipf_runs(1 << 16, key_dtype=np.int32)
    z2 = W.zipf_runs(1 << 16, key_dtype=np.uint64)
    # the int32 headline twin holds the same values as the uint64 workload
    assert np.array_equal(z1.keys.astype(np.uint64), z2.keys)
    assert z1.keys.min() >= 0 and z1.keys.max() < (1 << 20)


def test_batched_generator_does_not_depend_on_workers():
    one = W.batched_random_runs(nseg=24, lo_exp=4, hi_exp=12, workers=1)
    many = W.batched_random_runs(nseg=24, lo_exp=4, hi_exp=12, workers=3)
    assert np.array_equal(one.offsets, many.offsets)
    assert np.array_equal(one.keys, many.keys)
    sizes = np.diff(one.offsets.astype(np.int64))
    assert sizes.min() >= 16 and sizes.max() <= 4096
    # every segment is a permutation of 0..size-1 (random-runs model)
    for g in range(24):
        seg = one.keys[int(one.offsets[g]):int(one.offsets[g + 1])]
        assert np.array_equal(np.sort(seg), np.arange(seg.size))


def test_request_trace_shape():
    metas = W.trace_meta(rate_hz=2000.0, duration_s=0.05)
    arr = np.array([m.arrival_s for m in metas])
    assert np.all(np.diff(arr) >= 0) and arr.max() < 0.05
    sizes = np.array([m.n for m in metas])
    assert sizes.min() >= (1 << 12) and sizes.max() <= (1 << 24)
    assert {m.dtype for m in metas} <= {np.dtype(np.int32), np.dtype(np.int64), np.dtype(np.float32)}
    # about rate * duration arrivals (Poisson: 100 expected)
    assert 60 <= len(metas) <= 140


def test_request_pool_and_in_place_batches():
    # buffers are handed out back to back; a batch is sorted in place only
    # when it is consecutive requests of one pool
    import torch
    from paper_1805_04154_amd.serving import RequestPool, ServedRequest, SortServer
    pool = RequestPool(torch.int32, 100, device="cpu")
    a, b, c = pool.request(0, 0.0, 30), pool.request(1, 0.0, 50), pool.request(2, 0.0, 20)
    assert (a.offset, b.offset, c.offset) == (0, 30, 80) and pool.used == 100
    b.keys.fill_(7)
    assert int(pool.keys[30:80].sum()) == 7 * 50  # views of the pool's storage
    with pytest.raises(ValueError):
        pool.request(3, 0.0, 1)
    assert SortServer._in_place([a, b, c]) and SortServer._in_place([b]) and SortServer._in_place([b, c])
    assert not SortServer._in_place([a, c])  # a gap
    assert not SortServer._in_place([b, a])  # out of order
    other = RequestPool(torch.int32, 10, device="cpu").request(0, 0.0, 10)
    assert not SortServer._in_place([c, other])
    own = ServedRequest(9, 0.0, torch.zeros(5, dtype=torch.int32), torch.zeros(5, dtype=torch.int32))
    assert not SortServer._in_place([own]) and not SortServer._in_place([a, own])
    pool.reset()
    assert pool.request(4, 0.0, 100).offset == 0


def test_busy_time_is_the_union_of_intervals():
    from paper_1805_04154_amd.serving import busy_time
    assert busy_time([]) == 0.0
    assert busy_time([(0.0, 1.0)]) == 1.0
    assert busy_time([(0.0, 1.0), (0.5, 2.0)]) == 2.0  # overlap counted once
    assert busy_time([(3.0, 4.0), (0.0, 1.0)]) == 2.0  # disjoint, any order
    assert busy_time([(0.0, 5.0), (1.0, 2.0), (6.0, 7.0)]) == 6.0  # nested


def test_autotuner_search_space():
    pytest.importorskip("torch")
    from paper_1805_04154_amd import autotune
    from paper_1805_04154_amd.binding import TUNING_FIELDS
    full, small = autotune.candidates(), autotune.candidates(small=True)
    for cands in (full, small):
        keys = [tuple(sorted(c.items())) for c in cands]
        assert len(set(keys)) == len(keys)
        for c in cands:
            assert set(c) <= set(TUNING_FIELDS)
            assert c["merge_tile"] in (2048, 4096, 8192)
            assert c["merge_levels"] in (1, 2)
            assert all(1 <= c[k] <= 65536 for k in c if k.startswith("grid_"))
    import torch
    assert autotune.signature(3 << 20, 4096, torch.int32, None) == autotune.signature(2 << 20, 5000, torch.int32, 24)
    assert autotune.signature(1 << 20, 1, torch.int32, None) != autotune.signature(1 << 21, 1, torch.int32, None)


def pass_bound(n: int, w: int) -> int:
    """Largest merge pass the library launches for n keys at minimum run w:
    the smallest l >= 1 with 2^l (w + 1) >= 2n, capped at floor(lg n) + 1."""
    b = 1
    while (1 << b) * (w + 1) < 2 * n:
        b += 1
    return min(b, max(n, 1).bit_length())


def fused_pass_bound(n: int, fuse: int = 4096) -> int:
    """Largest power of a node of more than ``fuse`` elements: its internal
    boundaries have powers >= p, so its leaf midpoints share one cell of
    width 2^(1-p) and each leaf is shorter than n 2^(2-p); its size is below
    3n / 2^(p-1).  The smallest p with fuse 2^p >= 3n."""
    p = 1
    while (fuse << p) < 3 * n:
        p += 1
    return p


@pytest.mark.parametrize("w", [1, 24, 64])
def test_nodes_above_the_fused_size_are_within_the_fused_pass_bound(w):
    # merge passes above this bound would hold only nodes of at most 4096
    # elements, which merge inside fused subtrees, so the library skips them
    import math
    import oracle
    rng = W.make_rng(78)
    worst = 0
    for n in (5000, 9000, 50001, 300000, 1 << 20):
        inputs = [W.random_permutation(rng, n), rng.integers(0, 5, size=n),
                  W.random_runs(rng, n, max(2.0, math.sqrt(n)), 0.25), W.random_runs(rng, n, 40.0, 0.25),
                  W.random_runs(rng, n, 3000.0, 0.1)]
        for v in inputs:
            ref = oracle.powersort(np.asarray(v).astype(np.int32), None, min_run=w)
            starts = ref.starts.astype(np.int64)
            at = {int(s): j for j, s in enumerate(starts)}
            for lo, mid, hi in ref.merges.astype(np.int64):
                if hi - lo > 4096:
                    pw = int(ref.powers[at[int(mid)] - 1])
                    assert pw <= fused_pass_bound(n), (n, w, lo, mid, hi, pw)
                    worst = max(worst, fused_pass_bound(n) - pw)
    assert worst >= 0
    assert fused_pass_bound(1 << 28) == 18 and fused_pass_bound(3 << 10) == 2


@pytest.mark.parametrize("w", [1, 2, 3, 7, 24, 64])
def test_every_node_power_is_within_the_pass_bound(w):
    # the library runs merge passes pmax..1 only; a node above the bound
    # would never merge, so the oracle's powers must all lie within it
    import math
    import oracle
    rng = W.make_rng(77)
    for n in (2, 3, 5, 24, 25, 26, 49, 100, 1000, 4097, 20000):
        for v in (W.random_permutation(rng, n), rng.integers(0, 3, size=n), np.arange(n)[::-1].copy(),
                  W.random_runs(rng, n, max(2.0, math.sqrt(n)), 0.25)):
            ref = oracle.powersort(np.asarray(v).astype(np.int32), None, min_run=w)
            if ref.powers.size:
                assert int(ref.powers.max()) <= pass_bound(n, w), (n, w)
    # and the bound is attained up to one level on a permutation
    ref = oracle.powersort(W.random_permutation(rng, 1 << 16).astype(np.int32), None, min_run=w)
    assert int(ref.powers.max()) >= pass_bound(1 << 16, w) - 1


def fused_units(starts: np.ndarray, merges: np.ndarray, n: int, fuse: int = 4096):
    """Fused subtrees from the oracle's merge tree: the children of at most
    ``fuse`` elements of nodes larger than that (and the whole array if it
    is that small), as (elements, leaves)."""
    s = starts.astype(np.int64)
    leaves = lambda lo, hi: int(np.searchsorted(s, hi) - np.searchsorted(s, lo))
    out = []
    for lo, mid, hi in merges.astype(np.int64):
        if hi - lo > fuse:
            for a, b in ((lo, mid), (mid, hi)):
                if b - a <= fuse:
                    out.append((int(b - a), leaves(a, b)))
    if n <= fuse and n > 0:
        out.append((n, len(s) - 1))
    return out


@pytest.mark.parametrize("w", [1, 24, 64])
def test_fused_subtree_lists_fit_their_capacities(w):
    # The workspace holds one list per kernel that forms fused subtrees:
    # single natural runs longer than any min-run (at most n / 65 + 1 of
    # them), subtrees of eight or more leaves (at most r1 / 8 + 1) and the
    # rest (at most r1), with r1 = rmax + 1 and rmax = n / max(w, 2) + 2 the
    # leaf bound of the layout for one segment.
    import math
    import oracle
    rng = W.make_rng(79)
    seen = {"copy": 0, "few": 0, "radix": 0}
    for n in (70, 4096, 5000, 50001, 300000):
        for v in (W.random_permutation(rng, n), W.random_runs(rng, n, 40.0, 0.25),
                  W.random_runs(rng, n, max(2.0, math.sqrt(n)), 0.25), W.random_runs(rng, n, 3000.0, 0.1),
                  np.arange(n)[::-1].copy()):
            ref = oracle.powersort(np.asarray(v).astype(np.int32), None, min_run=w)
            rmax = min(n, n // max(w, 2) + 2)
            r1 = rmax + 1
            caps = {"copy": min(r1, n // 65 + 1), "radix": r1 // 8 + 1, "few": r1}
            count = {"copy": 0, "few": 0, "radix": 0}
            for size, nl in fused_units(ref.starts, ref.merges, n):
                kind = "copy" if (nl == 1 and size > 64) else ("radix" if nl >= 8 else "few")
                count[kind] += 1
            for k in count:
                assert count[k] <= caps[k], (n, w, k, count[k], caps[k])
                seen[k] += count[k]
    assert all(seen[k] > 0 for k in seen)  # every kind occurs


def test_arena_allocator_first_fit_and_coalescing():
    from paper_1805_04154_amd.serving import ALIGN, ArenaAllocator
    a = ArenaAllocator(10 * ALIGN)
    x = a.alloc(3 * ALIGN)
    y = a.alloc(ALIGN + 1)        # rounded up to 2 units
    z = a.alloc(4 * ALIGN)
    assert (x, y, z) == (0, 3 * ALIGN, 5 * ALIGN)
    assert a.in_use == 9 * ALIGN and a.largest_free() == ALIGN
    assert a.alloc(2 * ALIGN) is None  # one unit left
    a.release(y, ALIGN + 1)
    assert a.largest_free() == 2 * ALIGN and a.alloc(2 * ALIGN) == 3 * ALIGN
    a.release(3 * ALIGN, 2 * ALIGN)
    a.release(x, 3 * ALIGN)            # coalesces with the freed block on its right
    assert a.free[0] == (0, 5 * ALIGN)
    a.release(z, 4 * ALIGN)            # and everything merges back into one block
    assert a.free == [(0, 10 * ALIGN)] and a.in_use == 0
    with pytest.raises(ValueError):
        a.release(0, ALIGN)            # not allocated
