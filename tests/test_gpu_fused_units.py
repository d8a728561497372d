"""Fused subtrees of at most 4096 elements (single natural runs, subtrees of
few leaves, subtrees of many leaves) formed by blocks that take many
subtrees in turn, so that each block's loads of the next subtree overlap the
current one.  A tiny fused grid forces long chains of subtrees per block;
every key type, with and without a payload, is compared with the oracle
(keys bit for bit, payload order and merge cost)."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

N = (1 << 20) + 12345  # ragged: not a multiple of any tile
DTYPES = [np.int32, np.uint32, np.float32, np.int64, np.uint64]


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    binding.set_tuning(None)
    yield binding
    binding.set_tuning(None)


def make_keys(dtype, mean_run: float, seed: int) -> np.ndarray:
    """Random runs (a quarter decreasing) over values with repeats, so that
    equal keys test stability, cast to the key type with negatives where the
    type has them."""
    v = W.random_runs(np.random.default_rng(seed), N, mean_run, 0.25) // 3
    if dtype == np.int32:
        return (v - N // 6).astype(np.int32)
    if dtype == np.uint32:
        return (v * 4099).astype(np.uint32)
    if dtype == np.float32:
        return ((v - N // 6) * 0.5).astype(np.float32)  # exact: |v| < 2^20
    if dtype == np.int64:
        return (v - N // 6).astype(np.int64) * (1 << 33) + 7
    return v.astype(np.uint64) << np.uint64(30)


@pytest.mark.parametrize("dtype", DTYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("with_payload", [True, False], ids=["payload", "keys_only"])
@pytest.mark.parametrize("mean_run,grid", [(600.0, 3), (40.0, 5), (600.0, 97)], ids=["few_g3", "many_g5", "few_g97"])
def test_fused_subtrees_many_per_block(ps, dtype, with_payload, mean_run, grid):
    import torch
    import oracle
    keys = make_keys(dtype, mean_run, seed=int(mean_run) + grid)
    pay = np.arange(N, dtype=np.uint32)[::-1].copy()
    ref = oracle.powersort(keys, pay if with_payload else None, min_run=24)
    try:
        ps.set_tuning({"grid_fused": grid})
        k = to_dev(keys)
        p = to_dev(pay) if with_payload else None
        M = torch.zeros(1, dtype=torch.int64, device="cuda")
        ps.sort(k, p, merge_cost=M)
        torch.cuda.synchronize()
    finally:
        ps.set_tuning(None)
    got = to_host(k, dtype)
    assert np.array_equal(got.view(np.uint8), ref.keys.view(np.uint8)), "keys differ"
    if with_payload:
        assert np.array_equal(to_host(p, np.uint32), ref.payload), "payload order differs"
    assert int(M.item()) == ref.merge_cost
