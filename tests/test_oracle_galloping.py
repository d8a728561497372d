"""Pins of the oracle's galloping merge (the comparison-saving merge of
Timsort, described in Sec. 4.1 and named as future work in Sec. 5).

Galloping changes how a merge finds its output order, never the order:
  * results, payload order and merge cost equal the plain oracle's and the
    library stable sort, for every key type;
  * every comparison-based merge of runs of a and b elements needs at least
    lg C(a + b, a) comparisons on some input, and run detection compares each
    adjacent pair once, so a whole sort makes at least (n - 1) + sum over its
    merges of lg C(a + b, a) comparisons on inputs without further structure
    (checked on random permutations with w = 1, where no insertion sort runs);
  * a merge whose output alternates between the runs one element at a time
    never reaches the galloping threshold: its comparisons are the plain
    merge's exactly;
  * a merge whose output takes k blocks of L elements from alternate runs
    costs at most 7 comparisons before galloping starts and, per block, one
    exponential-plus-binary search over at most L + 1 positions, i.e. at most
    2 ceil(lg(L + 2)) + 2 comparisons; the plain merge needs about k L.
"""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W


def lg_binom(a: int, b: int) -> float:
    return (math.lgamma(a + b + 1) - math.lgamma(a + 1) - math.lgamma(b + 1)) / math.log(2)


def test_same_result_and_merge_cost_as_plain(oracle_mod):
    rng = W.make_rng(501)
    for n in (0, 1, 2, 50, 1000, 30_000):
        for w in (1, 24):
            for v in (rng.permutation(n), rng.integers(0, 4, size=n), W.random_runs(rng, n, max(2.0, n ** 0.5), 0.25),
                      np.arange(n)[::-1]):
                k = np.asarray(v).astype(np.int32)
                p = np.arange(n, dtype=np.uint32)
                a = oracle_mod.powersort(k, p, min_run=w)
                g = oracle_mod.powersort(k, p, min_run=w, galloping=True)
                order = np.argsort(k, kind="stable")
                assert np.array_equal(g.keys, k[order]) and np.array_equal(g.payload, p[order]), (n, w)
                assert g.merge_cost == a.merge_cost and np.array_equal(g.merges, a.merges), (n, w)
    for dt in (np.uint32, np.int64, np.uint64):
        k = rng.integers(0, 40, size=5000).astype(dt)
        assert np.array_equal(oracle_mod.powersort(k, galloping=True).keys, np.sort(k, kind="stable"))
    f = W.f32_from_values(rng, rng.permutation(3000), 3000)
    gp = oracle_mod.powersort(f, np.arange(3000, dtype=np.uint32), galloping=True).payload
    u = f.view(np.uint32)
    tot = np.where(u >> 31 == 1, ~u, u | np.uint32(0x80000000))
    assert np.array_equal(gp, np.argsort(tot, kind="stable").astype(np.uint32))


def test_information_lower_bound(oracle_mod):
    rng = W.make_rng(502)
    for n in (100, 5000, 200_000):
        k = rng.permutation(n).astype(np.int32)
        g = oracle_mod.powersort(k, min_run=1, galloping=True)
        m = g.merges.astype(np.int64)
        bound = (n - 1) + sum(lg_binom(int(mid - lo), int(hi - mid)) for lo, mid, hi in m)
        assert g.comparisons >= bound, (n, g.comparisons, bound)


def two_runs(left: np.ndarray, right: np.ndarray) -> np.ndarray:
    """Keys whose w = 1 partition is exactly the runs left and right (both
    ascending, with a descent where they meet)."""
    assert left[-1] > right[0]
    return np.concatenate([left, right]).astype(np.int32)


def test_alternating_merge_equals_plain(oracle_mod):
    for m in (10, 1000, 50_000):
        k = two_runs(np.arange(0, 2 * m, 2), np.arange(1, 2 * m, 2))  # output alternates left, right, ...
        a = oracle_mod.powersort(k, min_run=1)
        g = oracle_mod.powersort(k, min_run=1, galloping=True)
        assert a.r == 2 and g.comparisons == a.comparisons


@pytest.mark.parametrize("L,k", [(8, 20), (100, 50), (5000, 8), (100_000, 3)])
def test_block_merges_cost_logarithmic_per_block(oracle_mod, L, k):
    # block b (0..k-1) holds keys [b L, (b+1) L); even blocks form the left run
    blocks = [np.arange(b * L, (b + 1) * L) for b in range(k)]
    left = np.concatenate(blocks[0::2])
    right = np.concatenate(blocks[1::2])
    keys = two_runs(left, right)
    n = keys.shape[0]
    a = oracle_mod.powersort(keys, min_run=1)
    g = oracle_mod.powersort(keys, min_run=1, galloping=True)
    assert a.r == 2 and np.array_equal(g.keys, np.sort(keys))
    merge_plain, merge_gallop = a.comparisons - (n - 1), g.comparisons - (n - 1)
    assert merge_plain >= (k - 1) * L  # every element but the last block's is compared
    assert merge_gallop <= 7 + k * (2 * math.ceil(math.log2(L + 2)) + 2), (merge_gallop, merge_plain)


def test_one_run_before_the_other(oracle_mod):
    # every right element precedes every left one: the plain merge compares
    # each of the b right elements once; galloping stops after a few
    for a_len, b_len in ((10, 100_000), (100_000, 10), (5000, 5000)):
        keys = two_runs(np.arange(b_len, b_len + a_len), np.arange(b_len))
        n = a_len + b_len
        a = oracle_mod.powersort(keys, min_run=1)
        g = oracle_mod.powersort(keys, min_run=1, galloping=True)
        assert a.comparisons - (n - 1) == b_len
        assert g.comparisons - (n - 1) <= 7 + 2 + 2 * math.ceil(math.log2(b_len + 2)) + 2
