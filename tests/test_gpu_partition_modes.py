"""The leaf partition follows its chain through a 4096-position tile in one of
four ways, chosen per tile from the tile's own data: a jump (the tile lies
inside one long run), a walk over at most 32 listed run changes and breaks,
an arithmetic progression of step w (every natural run shorter than w), or
pointer jumping over a per-position successor table.  Each input below is
built to put many tiles in one of those ways, plus tiles that mix them at
their seams; leaf starts (ps_inspect), sorted output and M must equal the
oracle's for every w."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

TILE = 4096


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    return binding


def runs_of(rng, n, length_lo, length_hi, desc_frac=0.3):
    """Concatenated natural runs with lengths in [length_lo, length_hi]."""
    parts, total = [], 0
    while total < n:
        m = int(rng.integers(length_lo, length_hi + 1))
        v = np.sort(rng.integers(0, 1 << 30, size=m))
        if rng.random() < desc_frac:
            v = np.unique(v)[::-1]
        parts.append(v)
        total += len(v)
    return np.concatenate(parts)[:n]


def mode_inputs(rng):
    n = 9 * TILE + 123  # several tiles and a ragged tail
    yield "jump", runs_of(rng, n, 3 * TILE, 6 * TILE)
    yield "walk", runs_of(rng, n, 300, 1500)
    yield "dense", W.random_permutation(rng, n)
    yield "table", runs_of(rng, n, 70, 110)  # runs longer than w, too many to list
    yield "mixed", np.concatenate([runs_of(rng, 2 * TILE, 3 * TILE, 4 * TILE), W.random_permutation(rng, 2 * TILE),
                                   runs_of(rng, 2 * TILE, 70, 110), runs_of(rng, 2 * TILE + 77, 500, 900)])


@pytest.mark.parametrize("w", [2, 3, 24, 64])
def test_partition_modes_match_oracle(ps, w):
    import torch
    import oracle
    rng = W.make_rng(900 + w)
    for name, v in mode_inputs(rng):
        keys = np.asarray(v).astype(np.int32)
        ref = oracle.powersort(keys, np.arange(len(keys), dtype=np.uint32), min_run=w)
        got = ps.inspect(to_dev(keys), min_run=w)
        torch.cuda.synchronize()
        assert got["r"] == ref.r, (name, w)
        assert np.array_equal(got["starts"].cpu().numpy().astype(np.int64), ref.starts.astype(np.int64)), (name, w)
        k, p = to_dev(keys), to_dev(np.arange(len(keys), dtype=np.uint32))
        M = torch.zeros(1, dtype=torch.int64, device="cuda")
        ps.sort(k, p, min_run=w, merge_cost=M)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(k, np.int32), ref.keys), (name, w)
        assert np.array_equal(to_host(p, np.uint32), ref.payload), (name, w)
        assert int(M.item()) == ref.merge_cost, (name, w)


def test_partition_modes_segmented(ps):
    # segment starts are breaks: they push tiles out of the jump and dense
    # ways and into walk or table ones
    import torch
    import oracle
    rng = W.make_rng(950)
    parts = [v for _, v in mode_inputs(rng)]
    cuts = []
    for v in parts:  # split each input into a few segments at random places
        c = np.sort(rng.integers(0, len(v), size=3))
        cuts.extend(np.split(np.asarray(v), c))
    sizes = [len(c) for c in cuts]
    offsets = np.zeros(len(cuts) + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
    keys = np.concatenate(cuts).astype(np.int32)
    pay = np.arange(len(keys), dtype=np.uint32)
    rk, rp, rc = oracle.segmented_powersort(keys, pay, offsets)
    k, p = to_dev(keys), to_dev(pay)
    off = torch.from_numpy(offsets.view(np.int64)).cuda()
    costs = torch.zeros(len(cuts), dtype=torch.int64, device="cuda")
    ps.segmented_sort(k, p, off, merge_costs=costs)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(k, np.int32), rk)
    assert np.array_equal(to_host(p, np.uint32), rp)
    assert np.array_equal(costs.cpu().numpy().view(np.uint64), rc)
