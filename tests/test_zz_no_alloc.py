"""ps_sort_no_alloc (the sort in the library's fixed device scratch) against
ps_sort, through the C ABI: keys, payload and merge cost bit-identical on
consecutive calls, the second smaller than the first, for several key types
and options; no device memory is allocated by a call; inputs beyond the fixed
scratch are refused before anything is launched."""
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


def both(ps, keys, payload, **kw):
    """(keys, payload, M) from ps_sort and from ps_sort_no_alloc on copies."""
    import torch
    out = []
    for fn in (ps.sort, ps.sort_no_alloc):
        k = to_dev(keys)
        p = to_dev(payload) if payload is not None else None
        M = torch.zeros(1, dtype=torch.int64, device="cuda")
        fn(k, p, merge_cost=M, **kw)
        torch.cuda.synchronize()
        out.append((to_host(k, keys.dtype), None if p is None else to_host(p, np.uint32), int(M.item())))
    return out


def test_no_alloc_equals_sort_on_consecutive_calls(ps):
    import oracle
    print("no-alloc sort: int32 runs, 4.2M then 1M keys", flush=True)
    for n in ((1 << 22) + 12345, (1 << 20) - 3):  # the second call is smaller
        wl = W.runs_2p20(n=n)
        (k0, p0, m0), (k1, p1, m1) = both(ps, wl.keys, wl.payload)
        assert np.array_equal(k0, k1) and np.array_equal(p0, p1) and m0 == m1, n
        ref = oracle.powersort(wl.keys, wl.payload, details=False)
        assert np.array_equal(k1, ref.keys) and np.array_equal(p1, ref.payload) and m1 == ref.merge_cost


@pytest.mark.parametrize("dtype", [np.int64, np.float32, np.uint64])
def test_no_alloc_other_key_types(ps, dtype):
    print(f"no-alloc sort: {np.dtype(dtype).name}", flush=True)
    rng = W.make_rng(5)
    for n in (3_000_001, 65_537):
        vals = W.random_runs(rng, n, 1000.0, 0.25)
        keys = (W.f32_from_values(rng, vals, n) if dtype == np.float32
                else (vals.astype(np.int64) - n // 2).astype(dtype))
        (k0, p0, m0), (k1, p1, m1) = both(ps, keys, W.payload_for(n))
        assert np.array_equal(k0.view(np.uint8), k1.view(np.uint8)) and np.array_equal(p0, p1) and m0 == m1


def test_no_alloc_options_and_no_payload(ps):
    print("no-alloc sort: options", flush=True)
    wl = W.runs_2p20(n=(1 << 21) + 77)
    for kw in ({"min_run": 7}, {"method": "peeksort"}, {"compact_scratch": True}):
        (k0, p0, m0), (k1, p1, m1) = both(ps, wl.keys, wl.payload, **kw)
        assert np.array_equal(k0, k1) and np.array_equal(p0, p1) and m0 == m1, kw
    (k0, _, m0), (k1, _, m1) = both(ps, wl.keys, None)
    assert np.array_equal(k0, k1) and m0 == m1
    for n in (0, 1, 2):
        (k0, p0, m0), (k1, p1, m1) = both(ps, wl.keys[:n].copy(), W.payload_for(n))
        assert np.array_equal(k0, k1) and np.array_equal(p0, p1) and m0 == m1 == 0


def test_no_alloc_allocates_nothing_and_refuses_oversized(ps):
    import torch
    print("no-alloc sort: device memory and limits", flush=True)
    wl = W.runs_2p20(n=4_000_000)
    k = to_dev(wl.keys)
    p = to_dev(wl.payload)
    M = torch.zeros(1, dtype=torch.int64, device="cuda")
    ps.sort_no_alloc(k, p, merge_cost=M)  # the library's module is loaded by now
    torch.cuda.synchronize()
    k.copy_(to_dev(wl.keys))
    torch.cuda.synchronize()
    def fresh_stream():
        # A stream the library has no pool entry for, on which the runtime's
        # own set-up is already behind us: the first dispatch on a stream
        # sets up its hardware queue and, for kernels that spill registers,
        # that queue's per-lane scratch (runtime memory, not the library's).
        st = torch.cuda.Stream()
        k.copy_(src)
        torch.cuda.synchronize()
        ps.sort_no_alloc(k, p, merge_cost=M, stream=st)
        torch.cuda.synchronize()
        k.copy_(src)
        torch.cuda.synchronize()
        return st

    src = to_dev(wl.keys)
    s = fresh_stream()
    free0, _ = torch.cuda.mem_get_info()
    ps.sort_no_alloc(k, p, merge_cost=M, stream=s)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (4 << 20)
    assert bool((k[1:] >= k[:-1]).all())
    # the same measurement sees ps_sort's pool allocation (about 70 MiB here)
    s2 = fresh_stream()
    free2, _ = torch.cuda.mem_get_info()
    ps.sort(k, p, merge_cost=M, stream=s2)
    torch.cuda.synchronize()
    free3, _ = torch.cuda.mem_get_info()
    assert free2 - free3 > (48 << 20)
    ps.release(s2)
    big = torch.zeros(7_000_000, dtype=torch.int32, device="cuda")
    bp = torch.zeros(7_000_000, dtype=torch.int32, device="cuda")
    with pytest.raises(ps.PowersortError) as e:
        ps.sort_no_alloc(big, bp)
    assert e.value.status == -2
