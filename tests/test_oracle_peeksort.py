"""Pins of the peeksort oracle (Alg. PeekSort, Sec. 3.1) against what the
paper and mathematics fix: the Method 1 tree drawn in Fig. 1 (left), the
merge-cost bound of Thm. "peeksort", an independent formulation of the split
rule (the run boundary nearest to the range midpoint), a library stable
sort, and the leaf partition shared with powersort."""
import json
import math
import os

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
FIG1L = json.load(open(os.path.join(HERE, "golden", "fig1_peeksort.json")))


def entropy_bits(lengths):
    n = float(sum(lengths))
    return sum((L / n) * math.log2(n / L) for L in lengths)


def nearest_boundary_tree(lengths):
    """Method 1 written independently: a range of runs with elements
    [lo, hi) splits at the interior run boundary b nearest to
    lo + floor((hi - 1 - lo) / 2) + 1/2, the larger b on a tie.  Returns the
    set of (lo, mid, hi) and the leaf depths."""
    S = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    merges, depth = set(), [0] * len(lengths)

    def rec(a, b, d):
        if b - a == 1:
            depth[a] = d
            return
        lo, hi = int(S[a]), int(S[b])
        target2 = 2 * (lo + (hi - 1 - lo) // 2) + 1  # twice the midpoint m + 1/2
        best = None
        for c in range(a + 1, b):
            dist = abs(2 * int(S[c]) - target2)
            if best is None or dist < best[0] or (dist == best[0] and c > best[1]):
                best = (dist, c)
        c = best[1]
        merges.add((lo, int(S[c]), hi))
        rec(a, c, d + 1)
        rec(c, b, d + 1)

    if len(lengths):
        rec(0, len(lengths), 0)
    return merges, depth


def test_fig1_left_tree(oracle_mod):
    merges, depth, M = oracle_mod.peek_merge_order(FIG1L["run_lengths"])
    assert M == FIG1L["merge_cost"] == 65
    assert depth.tolist() == FIG1L["leaf_depths"]
    assert {tuple(int(v) for v in m) for m in merges} == {tuple(m) for m in FIG1L["merges_lo_mid_hi_0based"]}
    # post-order: every merge comes after the merges of its two parts
    seen = set()
    for lo, mid, hi in merges.tolist():
        for part in ((lo, mid), (mid, hi)):
            inner = [m for m in merges.tolist() if (m[0], m[2]) == part]
            assert all(tuple(x) in seen for x in inner)
        seen.add((lo, mid, hi))


@pytest.mark.parametrize("seed", range(6))
def test_split_rule_matches_nearest_boundary(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    for _ in range(300):
        r = int(rng.integers(1, 40))
        hi = int(rng.choice([2, 4, 30, 1000]))  # small lengths produce ties
        L = rng.integers(1, hi, size=r)
        merges, depth, M = oracle_mod.peek_merge_order(L)
        ref, ref_depth = nearest_boundary_tree(L.tolist())
        assert {tuple(int(v) for v in m) for m in merges} == ref
        assert depth.tolist() == ref_depth
        assert M == sum(d * int(x) for d, x in zip(ref_depth, L))


def test_tie_goes_to_the_right_boundary(oracle_mod):
    # runs 1,3,1 (n = 5): m = 2 lies in run [1..3] with m - i = 1 = j - m, a
    # tie, so the cut is after that run (at 4), not before it (at 1)
    merges, _, M = oracle_mod.peek_merge_order([1, 3, 1])
    got = {tuple(int(v) for v in m) for m in merges}
    assert (0, 4, 5) in got and (0, 1, 4) in got and M == 9
    # runs 2,2,2,2 (n = 8): m = 3 in run [2..3], m - i = 1 > 0 = j - m: cut at 4
    merges, _, M = oracle_mod.peek_merge_order([2, 2, 2, 2])
    assert M == 16 and (0, 4, 8) in {tuple(int(v) for v in m) for m in merges}
    # runs 1,2,1 (n = 4): m = 1 in run [1..2], m - i = 0 < 1 = j - m: cut at 1
    merges, _, _ = oracle_mod.peek_merge_order([1, 2, 1])
    assert (0, 1, 4) in {tuple(int(v) for v in m) for m in merges}


def test_merge_cost_bound_of_theorem(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(400):
        r = int(rng.integers(2, 300))
        L = rng.integers(1, int(rng.choice([3, 50, 5000])), size=r)
        n = int(L.sum())
        _, _, M = oracle_mod.peek_merge_order(L)
        H = entropy_bits(L.tolist())
        assert M <= H * n + 2 * n - (r + 2) + 1e-6 * n
        assert M >= H * n - 1e-6 * n  # no binary merge tree beats the entropy


def test_depth_stays_within_twice_lg_n(oracle_mod):
    """The bound that sizes the GPU's level loop: a node at depth d + 2 covers
    at most half of its ancestor at depth d, so leaves sit at depth
    <= 2 floor(lg n) (internal nodes one less)."""
    rng = np.random.default_rng(5)
    families = [
        [2 ** i for i in range(20)],                 # geometric
        [2 ** i for i in range(20)][::-1],
        [1, 10 ** 6] * 40,                           # huge runs between singletons
        [3 ** i for i in range(12)] + [1] * 50,
        list(rng.integers(1, 4, size=3000)),
        [int(x) for x in np.floor(1.6 ** np.arange(30))],
    ]
    for t in range(3000):
        r = int(rng.integers(2, 50))
        kind = t % 4
        if kind == 0:
            L = rng.integers(1, 4, r)
        elif kind == 1:
            L = (2.0 ** rng.uniform(0, 12, r)).astype(np.int64) + 1
        elif kind == 2:
            L = np.array([1 if i % 2 else int(rng.integers(1, 5000)) for i in range(r)])
        else:
            L = rng.permutation(np.array([int(1.7 ** i) + 1 for i in range(r)]))
        families.append([int(x) for x in L])
    for L in families:
        _, depth, _ = oracle_mod.peek_merge_order(L)
        n = int(sum(L))
        assert int(depth.max()) <= 2 * (n.bit_length() - 1), (L[:5], int(depth.max()))


@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.int64, np.uint64, np.float32])
def test_output_is_the_stable_sort(oracle_mod, dtype):
    rng = np.random.default_rng(3)
    for n in (0, 1, 2, 37, 1000, 5000):
        if dtype == np.float32:
            keys = rng.integers(-50, 50, size=n).astype(np.float32)
            if n > 10:
                keys[:6] = [np.inf, -np.inf, 0.0, -0.0, np.nan, -np.nan]
        else:
            info = np.iinfo(dtype)
            keys = rng.integers(max(info.min, -100), min(info.max, 100), size=n).astype(dtype)
        pay = np.arange(n, dtype=np.uint32)
        for w in (1, 24):
            res = oracle_mod.peeksort(keys, pay, min_run=w)
            if dtype == np.float32:
                u = keys.view(np.uint32)
                ordkey = np.where(u >> 31, ~u, u | np.uint32(0x80000000))
                ref = np.argsort(ordkey, kind="stable")
            else:
                ref = np.argsort(keys, kind="stable")
            assert np.array_equal(res.payload, ref.astype(np.uint32))
            assert np.array_equal(res.keys.view(np.uint8), keys[ref].view(np.uint8))


@pytest.mark.parametrize("w", [1, 3, 24])
def test_same_leaves_as_powersort_and_depth_sum(oracle_mod, w):
    wl = W.runs_2p20()
    keys, pay = wl.keys[:200000], wl.payload[:200000]
    pk = oracle_mod.peeksort(keys, pay, min_run=w)
    pw = oracle_mod.powersort(keys, pay, min_run=w)
    assert np.array_equal(pk.starts, pw.starts)
    L = np.diff(pk.starts.astype(np.int64))
    assert pk.merge_cost == int((pk.depth.astype(np.int64) * L).sum())
    assert sorted(map(tuple, pk.merges.tolist())) == sorted(nearest_boundary_tree(L.tolist())[0])
    assert np.array_equal(pk.keys, pw.keys) and np.array_equal(pk.payload, pw.payload)


def test_segmented_is_per_segment(oracle_mod):
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 40, size=3000).astype(np.int32)
    off = np.array([0, 0, 1, 700, 701, 2999, 3000], np.uint64)
    k, p, costs = oracle_mod.segmented_peeksort(keys, np.arange(3000, dtype=np.uint32), off)
    for g in range(len(off) - 1):
        a, b = int(off[g]), int(off[g + 1])
        one = oracle_mod.peeksort(keys[a:b], np.arange(a, b, dtype=np.uint32))
        assert np.array_equal(k[a:b], one.keys) and np.array_equal(p[a:b], one.payload)
        assert costs[g] == one.merge_cost
