"""Parity at the full sizes the benchmark runs, in its launch configuration
(default tuning, uint32 index payload, w = 24): every output key, the whole
payload permutation and the merge cost M against the oracle run on the same
input.  Large: these run the oracle on up to 2^28 keys (seconds each), and
one input of the largest supported size, 2^31 - 1 keys (about a minute)."""
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


def largest_input() -> np.ndarray:
    """2^31 - 1 int32 keys in nine runs of uneven lengths: ascending runs that
    repeat keys (ties decided by stability) and strictly descending runs
    (reversed), so positions, leaf starts and powers reach the top of the
    supported range."""
    n = (1 << 31) - 1
    lengths = [int(f * n) for f in (0.21, 0.05, 0.13, 0.02, 0.30, 0.07, 0.11, 0.04)]
    lengths.append(n - sum(lengths))
    parts = []
    for j, L in enumerate(lengths):
        t = np.arange(L, dtype=np.int64)
        v = 3 * (L - 1 - t) + j if j % 3 == 1 else (t * (j + 2)) // 7 + 11 * j
        parts.append(v.astype(np.int32))
        del t, v
    return np.concatenate(parts)


def test_largest_segment_2p31_minus_1(ps):
    import torch
    import oracle
    print("full-size parity: 2^31 - 1 int32 keys", flush=True)
    keys = largest_input()
    pay = np.arange(keys.shape[0], dtype=np.uint32)
    ref = oracle.powersort(keys, pay, details=False)
    k = torch.from_numpy(keys).cuda()
    p = torch.from_numpy(pay.view(np.int32)).cuda()
    del keys, pay
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ps.sort(k, p.view(torch.uint32), merge_cost=M)
    torch.cuda.synchronize()
    assert int(M.item()) == ref.merge_cost
    assert np.array_equal(p.cpu().numpy().view(np.uint32), ref.payload)
    assert np.array_equal(k.cpu().numpy(), ref.keys)
    del k, p
    torch.cuda.empty_cache()
