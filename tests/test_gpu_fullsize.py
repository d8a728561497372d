"""Parity at the full sizes the benchmark runs, in its launch configuration
(default tuning, uint32 index payload, w = 24): every output key, the whole
payload permutation and the merge cost M against the oracle run on the same
input.  Large: these run the oracle on up to 2^28 keys (seconds each)."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_04154_amd import binding
    binding.load_library()
    binding.set_tuning(None)
    return binding


def full_check(ps, wl, method="powersort"):
    import torch
    import oracle
    print(f"full-size parity: {wl.name} ({method})", flush=True)
    ref = (oracle.powersort if method == "powersort" else oracle.peeksort)(wl.keys, wl.payload, details=False)
    k, p = to_dev(wl.keys), to_dev(wl.payload)
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ps.sort(k, p, merge_cost=M, method=method)
    torch.cuda.synchronize()
    assert int(M.item()) == ref.merge_cost
    assert np.array_equal(to_host(p, np.uint32), ref.payload)
    assert np.array_equal(to_host(k, wl.keys.dtype).view(np.uint8), ref.keys.view(np.uint8))
    del k, p
    torch.cuda.empty_cache()


def test_headline_zipf_int32_2p28(ps):
    full_check(ps, W.zipf_runs(1 << 28, key_dtype=np.int32))


def test_headline_zipf_int32_2p28_peeksort(ps):
    full_check(ps, W.zipf_runs(1 << 28, key_dtype=np.int32), method="peeksort")


def test_zipf_uint64_2p28(ps):
    full_check(ps, W.zipf_runs(1 << 28, key_dtype=np.uint64))


def test_permutation_2p26(ps):
    full_check(ps, W.permutation_i32(1 << 26))


def test_runs_2p26(ps):
    full_check(ps, W.runs_sqrt_i32(1 << 26))
