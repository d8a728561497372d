"""The merge-cost study (Sec. 4's input families) on the GPU: ps_merge_cost
for powersort and peeksort equals the oracle's M on every family, and for
the random-runs input of Sec. 4.3 it reproduces the printed average merge
cost 1.14e8 (the oracle pin ties the same input to that value)."""
import math

import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    return binding


FAMILIES = [
    ("permutation", lambda n: W.random_permutation(W.make_rng(51), n)),
    ("runs_sqrt", lambda n: W.random_runs(W.make_rng(52), n, math.sqrt(n), 0.0)),
    ("runs_64_rev", lambda n: W.random_runs(W.make_rng(53), n, 64.0, 0.25)),
    ("zipf", lambda n: W.zipf_runs(n, key_dtype=np.int32).keys),
]


@pytest.mark.parametrize("name,gen", FAMILIES)
@pytest.mark.parametrize("method", ["powersort", "peeksort"])
def test_family_merge_cost_matches_oracle(ps, name, gen, method):
    import torch
    import oracle
    keys = np.ascontiguousarray(gen(1 << 20)).astype(np.int32)
    ref = (oracle.powersort if method == "powersort" else oracle.peeksort)(keys, None, details=False)
    M = ps.merge_cost(torch.from_numpy(keys).cuda(), method=method)
    torch.cuda.synchronize()
    assert int(M.item()) == ref.merge_cost
    n = len(keys)
    assert ref.merge_cost <= n * math.log2(n) + 2 * n


def test_sec43_random_runs_cost(ps):
    import torch
    import oracle
    n = 10 ** 7
    keys = W.random_runs(W.make_rng(0), n, 3000.0, 0.0).astype(np.int32)
    M = int(ps.merge_cost(torch.from_numpy(keys).cuda()).item())
    assert M == oracle.powersort(keys, None, details=False).merge_cost
    assert abs(M / 1.14e8 - 1) < 0.015
