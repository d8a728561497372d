"""Pins of the oracle's elementary mergesorts (the top-down and bottom-up
mergesorts of the paper's experiments, Sec. 4.1 setup: a check before each
merge whether its runs are already in order, insertion sort below w).

Each pin is fixed by something other than the oracle's own loop:
  * the output is the unique stable sort (numpy's stable argsort);
  * sorted and all-equal inputs need no merge at all (M = 0);
  * on strictly decreasing input every check fails, so M equals the closed
    form of the non-adaptive recursion: top-down T(n) = n + T(ceil(n/2)) +
    T(floor(n/2)) above w, bottom-up the sum over run lengths m = w, 2w, ...
    of n minus a last run left without a partner, and n k for n = w 2^k;
  * on any input, a merge runs exactly when some key of its right part is
    below some key of its left part in the ORIGINAL data (its parts are sorted
    before the check, so the check compares the left maximum with the right
    minimum), evaluated here over the fixed recursion shapes with numpy.
"""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W

W_CUT = 24


def topdown_closed(n: int, w: int) -> int:
    if n <= w:
        return 0
    return n + topdown_closed((n + 1) // 2, w) + topdown_closed(n // 2, w)


def bottomup_closed(n: int, w: int) -> int:
    total, m = 0, w
    while m < n:
        blocks = -(-n // m)
        alone = (n - (blocks - 1) * m) if blocks % 2 else 0
        total += n - alone
        m *= 2
    return total


def topdown_nodes(n: int, w: int):
    """(lo, mid, hi) of every merge point of the top-down recursion shape."""
    out, stack = [], [(0, n)]
    while stack:
        lo, hi = stack.pop()
        if hi - lo <= w:
            continue
        mid = lo + (hi - lo + 1) // 2
        out.append((lo, mid, hi))
        stack += [(lo, mid), (mid, hi)]
    return out


def bottomup_nodes(n: int, w: int):
    out, m = [], w
    while m < n:
        lo = 0
        while lo + m < n:
            out.append((lo, lo + m, min(lo + 2 * m, n)))
            lo += 2 * m
        m *= 2
    return out


def cost_from_data(keys: np.ndarray, nodes) -> int:
    """Sum of hi - lo over the nodes whose right part holds a key below the
    largest key of their left part, in the original data."""
    return sum(hi - lo for lo, mid, hi in nodes if keys[mid:hi].min() < keys[lo:mid].max())


SORTS = ("topdown_mergesort", "bottomup_mergesort")


@pytest.mark.parametrize("name", SORTS)
def test_output_is_the_stable_sort(oracle_mod, name):
    rng = W.make_rng(301)
    for n in (0, 1, 2, 23, 24, 25, 49, 100, 1000, 4097):
        for w in (1, 3, 24):
            keys = rng.integers(0, max(2, n // 4), size=n).astype(np.int32)
            pay = np.arange(n, dtype=np.uint32)
            r = getattr(oracle_mod, name)(keys, pay, min_run=w)
            order = np.argsort(keys, kind="stable")
            assert np.array_equal(r.keys, keys[order]) and np.array_equal(r.payload, pay[order]), (n, w)
    # every key type, floats by total order
    f = W.f32_from_values(rng, rng.permutation(3000), 3000)
    r = getattr(oracle_mod, name)(f, np.arange(3000, dtype=np.uint32))
    u = f.view(np.uint32)
    tot = np.where(u >> 31 == 1, ~u, u | np.uint32(0x80000000))
    assert np.array_equal(r.payload, np.argsort(tot, kind="stable").astype(np.uint32))
    for dt in (np.int64, np.uint64, np.uint32):
        k = rng.integers(0, 50, size=777).astype(dt)
        assert np.array_equal(getattr(oracle_mod, name)(k).keys, np.sort(k, kind="stable"))


@pytest.mark.parametrize("name", SORTS)
def test_no_merge_on_inputs_already_in_order(oracle_mod, name):
    for n in (1, 24, 25, 1000, 5001):
        assert getattr(oracle_mod, name)(np.arange(n, dtype=np.int32)).merge_cost == 0
        assert getattr(oracle_mod, name)(np.full(n, 7, np.int32)).merge_cost == 0
    # two ascending halves that meet in equal keys are in order as well
    k = np.concatenate([np.arange(0, 600), np.arange(599, 1300)]).astype(np.int32)
    assert getattr(oracle_mod, name)(k).merge_cost == 0


@pytest.mark.parametrize("w", [1, 2, 5, 24])
def test_decreasing_input_costs_the_closed_forms(oracle_mod, w):
    for n in (w + 1, 50, 97, 128, 1000, 4099, 30000):
        k = np.arange(n, 0, -1).astype(np.int32)
        assert oracle_mod.topdown_mergesort(k, min_run=w).merge_cost == topdown_closed(n, w), (n, w)
        assert oracle_mod.bottomup_mergesort(k, min_run=w).merge_cost == bottomup_closed(n, w), (n, w)
    for kk in range(1, 8):
        n = w * (1 << kk)
        k = np.arange(n, 0, -1).astype(np.int32)
        assert oracle_mod.topdown_mergesort(k, min_run=w).merge_cost == n * kk
        assert oracle_mod.bottomup_mergesort(k, min_run=w).merge_cost == n * kk


@pytest.mark.parametrize("w", [1, 3, 24])
def test_merge_cost_recomputed_from_the_original_data(oracle_mod, w):
    rng = W.make_rng(302)
    for n in (7, 60, 1000, 10007):
        inputs = [rng.permutation(n), rng.integers(0, 4, size=n), W.random_runs(rng, n, math.sqrt(n), 0.25),
                  W.random_runs(rng, n, 40.0, 0.1), np.concatenate([np.arange(n // 2), np.arange(n - n // 2)])]
        for v in inputs:
            k = np.asarray(v).astype(np.int32)
            td = oracle_mod.topdown_mergesort(k, min_run=w).merge_cost
            bu = oracle_mod.bottomup_mergesort(k, min_run=w).merge_cost
            assert td == cost_from_data(k, topdown_nodes(n, w)), (n, w)
            assert bu == cost_from_data(k, bottomup_nodes(n, w)), (n, w)
            assert td <= topdown_closed(n, w) and bu <= bottomup_closed(n, w)
