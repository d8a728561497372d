"""Pins of the oracle's key-comparison counts (Thm. "powersort" and
"peeksort" bound them): exact counts on small hand-checked inputs, run
detection costing n - 1 comparisons plus each merge between min(a, b) and
a + b - 1, and the theorems' bounds H n + 3n - r (powersort) and
H n + 3n - (2r + 3) (peeksort) for pure natural runs (w = 1)."""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W


def entropy_bits(lengths):
    n = float(sum(lengths))
    return sum((L / n) * math.log2(n / L) for L in lengths)


@pytest.mark.parametrize("method", ["powersort", "peeksort"])
def test_exact_small_counts(oracle_mod, method):
    sort = getattr(oracle_mod, method)
    a = lambda v: np.array(v, dtype=np.int32)
    assert sort(a(range(10)), None, min_run=1).comparisons == 9               # one ascending run
    assert sort(a(range(10))[::-1].copy(), None, min_run=1).comparisons == 9  # one descending run
    # two runs of 3, interleaved: 5 for detection + 5 for the merge
    assert sort(a([1, 3, 5, 2, 4, 6]), None, min_run=1).comparisons == 10
    # two runs of 3, right one entirely smaller: 5 + 3
    assert sort(a([4, 5, 6, 1, 2, 3]), None, min_run=1).comparisons == 8
    assert sort(a([]), None, min_run=1).comparisons == 0
    assert sort(a([7]), None, min_run=1).comparisons == 0


@pytest.mark.parametrize("method", ["powersort", "peeksort"])
def test_detection_plus_merge_bounds(oracle_mod, method):
    rng = np.random.default_rng(8)
    sort = getattr(oracle_mod, method)
    for _ in range(60):
        n = int(rng.integers(2, 5000))
        keys = W.random_runs(rng, n, float(rng.choice([2.0, 20.0, 300.0])), 0.25).astype(np.int32)
        res = sort(keys, None, min_run=1)
        lo = hi = n - 1
        for m_lo, m_mid, m_hi in res.merges.astype(np.int64):
            a, b = m_mid - m_lo, m_hi - m_mid
            lo += min(a, b)
            hi += a + b - 1
        assert lo <= res.comparisons <= hi


@pytest.mark.parametrize("method", ["powersort", "peeksort"])
def test_theorem_comparison_bounds(oracle_mod, method):
    rng = np.random.default_rng(9)
    sort = getattr(oracle_mod, method)
    for _ in range(60):
        n = int(rng.integers(2, 20000))
        keys = W.random_runs(rng, n, float(rng.choice([2.0, 30.0, 1000.0])), 0.25).astype(np.int32)
        res = sort(keys, None, min_run=1)
        L = np.diff(res.starts.astype(np.int64))
        r = len(L)
        H = entropy_bits(L.tolist())
        bound = H * n + 3 * n - (r if method == "powersort" else 2 * r + 3)
        assert res.comparisons <= bound + 1e-6 * n, (n, r, res.comparisons, bound)
