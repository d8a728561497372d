"""Parity of ps_alphabetic_tree (Method 2' as a standalone nearly-optimal
alphabetic tree builder) with the oracle's merge order for the same leaf
weights: node powers, the tree (node leaf ranges), leaf depths and the
weighted path length, bit-exact; plus the status word for bad weights."""
import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import merges_from_ranges, oracle_leaf_depths

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    return binding


def run(ps, weights):
    import torch
    w = torch.from_numpy(np.ascontiguousarray(weights, dtype=np.int32)).cuda()
    out = ps.alphabetic_tree(w)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(ps, weights):
    import oracle
    weights = np.asarray(weights, dtype=np.int64)
    r = len(weights)
    got = run(ps, weights)
    assert int(got["status"][0]) == 0
    powers, merges, M = oracle.merge_order(weights)
    assert int(got["cost"][0]) == M
    assert np.array_equal(got["powers"][1:r], powers)
    assert got["powers"][0] == 0 and got["powers"][r] == 0
    starts = np.concatenate([[0], np.cumsum(weights)]).astype(np.int64)
    want = {tuple(int(x) for x in m) for m in merges}
    assert merges_from_ranges(starts, got["powers"], got["node_left"], got["node_right"]) == want
    assert np.array_equal(got["leaf_depth"].astype(np.int64), oracle_leaf_depths(starts.astype(np.uint64), merges))
    return got


def test_fig1_weights(ps):
    fig = json.load(open(os.path.join(HERE, "golden", "fig1_powersort.json")))
    got = check(ps, fig["run_lengths"])
    assert got["powers"][1:6].tolist() == fig["powers"]
    assert int(got["cost"][0]) == fig["merge_cost"]


@pytest.mark.parametrize("seed", range(4))
def test_random_weights(ps, seed):
    rng = np.random.default_rng(seed)
    for r in (1, 2, 3, 17, 1000, 4097, 70000):
        hi = int(rng.choice([2, 30, 5000]))
        check(ps, rng.integers(1, hi, size=r))


def test_large_and_skewed(ps):
    rng = np.random.default_rng(7)
    check(ps, rng.integers(1, 2000, size=1 << 20))
    w = (2.0 ** rng.uniform(0, 20, size=5000)).astype(np.int64) + 1   # heavy-tailed weights
    check(ps, w)
    check(ps, [1 << 30, 1, 1, (1 << 30) - 10])                        # sum just below 2^31


def test_bad_weights_are_reported(ps):
    import oracle
    got = run(ps, [3, 0, 5, 2])
    assert int(got["status"][0]) == -1  # PS_ERR_INVALID_ARG: a zero weight
    _, _, M1 = oracle.merge_order(np.ones(4, np.int64))
    assert int(got["cost"][0]) == M1    # unit weights on error
    got = run(ps, [1 << 30, 1 << 30, 5])
    assert int(got["status"][0]) == -2  # PS_ERR_TOO_LARGE: sum >= 2^31
