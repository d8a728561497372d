"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/powersort_hip.h declares, and rejects bad arguments
before launching anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "powersort_hip.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1805_04154_amd import binding
    return binding.load_library()


def test_header_declares_the_binding_exports():
    from paper_1805_04154_amd import binding
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _opts(binding, min_run=0, flags=0, size=None):
    o = binding.PsOptions(size if size is not None else ctypes.sizeof(binding.PsOptions), min_run, flags, 0, None, 0)
    return ctypes.byref(o)


def test_argument_validation_without_launch(lib):
    from paper_1805_04154_amd import binding
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    assert lib.ps_sort(fake, None, 10, 0, _opts(binding, min_run=65), None, None) == -5
    assert b"min_run" in lib.ps_last_error()
    assert lib.ps_sort(fake, None, 10, 0, _opts(binding, flags=4), None, None) == -5  # unknown bit
    assert lib.ps_sort(fake, None, 10, 0, _opts(binding, flags=7), None, None) == -5
    assert lib.ps_sort(fake, None, 10, 0, _opts(binding, size=8), None, None) == -1
    assert lib.ps_sort(fake, None, 10, 7, None, None, None) == -1
    assert lib.ps_sort(None, None, 10, 0, None, None, None) == -1
    assert lib.ps_sort(fake, None, 1 << 31, 0, None, None, None) == -2
    assert lib.ps_segmented_sort(fake, None, None, 3, 10, 0, None, None, None, None) == -1
    assert lib.ps_segmented_sort(fake, None, fake, 0, 10, 0, None, None, None, None) == -1
    # a segmented batch may hold up to 2^63 - 1 keys in all (chunked above
    # 2^31 - 1); one array stays below 2^31
    assert lib.ps_segmented_sort(fake, None, fake, 2, 1 << 63, 0, None, None, None, None) == -2
    assert b"2^63" in lib.ps_last_error()
    assert lib.ps_segmented_merge_cost(fake, fake, 2, 1 << 63, 0, None, fake, None, None) == -2
    assert lib.ps_inspect(fake, fake, 2, 1 << 31, 0, None, ctypes.byref(binding.PsInspectOut()), None) == -2
    assert lib.ps_merge_cost(fake, 1 << 31, 0, None, fake, None) == -2
    assert lib.ps_workspace_bytes(1 << 31, 1, 0, 1, None) == 0
    assert lib.ps_workspace_bytes((1 << 31) - 1, 2, 0, 1, None) > 0
    # above 2^31 - 1 keys the batch runs in chunks below 2^31: the workspace
    # is that of the largest possible chunk
    assert lib.ps_workspace_bytes(1 << 31, 2, 0, 1, None) == lib.ps_workspace_bytes((1 << 31) - 1, 2, 0, 1, None)
    assert lib.ps_workspace_bytes(1 << 40, 2, 0, 1, None) == lib.ps_workspace_bytes((1 << 31) - 1, 2, 0, 1, None)
    assert lib.ps_workspace_bytes(1 << 63, 2, 0, 1, None) == 0
    assert lib.ps_merge_cost(fake, 10, 0, None, None, None) == -1
    assert lib.ps_segmented_merge_cost(fake, fake, 2, 10, 0, None, None, None, None) == -1
    assert lib.ps_inspect(fake, None, 1, 10, 0, None, None, None) == -1
    assert lib.ps_alphabetic_tree(fake, 0, None, None, None, None, None, None, None) == -1
    assert lib.ps_alphabetic_tree(fake, (1 << 28) + 1, None, None, None, None, None, None, None) == -2
    assert lib.ps_alphabetic_tree(None, 5, None, None, None, None, None, None, None) == -1


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.ps_status_string(code).startswith(b"PS_")
    assert lib.ps_status_string(42) == b"unknown ps_status"


def test_workspace_bytes(lib):
    from paper_1805_04154_amd import binding
    small = lib.ps_workspace_bytes(1 << 20, 1, 0, 1, None)
    big = lib.ps_workspace_bytes(1 << 28, 1, 0, 1, None)
    wide = lib.ps_workspace_bytes(1 << 28, 1, 3, 1, None)
    nopay = lib.ps_workspace_bytes(1 << 28, 1, 0, 0, None)
    assert 0 < small < big < wide
    assert nopay < big
    # scratch for two copies of keys+payload plus metadata well below the data
    # size (the merge-tile records are sized by the bound M <= n (lg n + 2))
    assert 2 * (1 << 28) * 8 <= big < 2 * (1 << 28) * 8 * 1.4
    # PS_FLAG_COMPACT_SCRATCH: one copy
    compact = lib.ps_workspace_bytes(1 << 28, 1, 0, 1, _opts(binding, flags=2))
    assert big - compact == (1 << 28) * 8
    peek = lib.ps_workspace_bytes(1 << 28, 1, 0, 1, _opts(binding, flags=1))
    assert peek - lib.ps_workspace_bytes(1 << 28, 1, 0, 1, _opts(binding, flags=3)) == (1 << 28) * 8
    assert lib.ps_workspace_bytes(10, 0, 0, 1, None) == 0
    assert lib.ps_workspace_bytes(10, 1, 9, 1, None) == 0
    assert lib.ps_workspace_bytes(10, 1, 0, 1, _opts(binding, min_run=99)) == 0


def test_tuning_roundtrip_on_host():
    from paper_1805_04154_amd import binding
    binding.set_tuning(None)
    d = binding.get_tuning()
    assert d["merge_tile"] == 8192
    binding.set_tuning({"merge_tile": 2048, "grid_merge": 333})
    d2 = binding.get_tuning()
    assert d2["merge_tile"] == 2048 and d2["grid_merge"] == 333 and d2["grid_fused"] == d["grid_fused"]
    with pytest.raises(binding.PowersortError):
        binding.set_tuning({"merge_tile": 1000})
    with pytest.raises(binding.PowersortError):
        binding.set_tuning({"merge_tile": 16384})
    binding.set_tuning({"merge_tile": 8192})
    assert binding.get_tuning()["merge_tile"] == 8192
    with pytest.raises(binding.PowersortError):
        binding.set_tuning({"grid_split": 1 << 20})
    with pytest.raises(binding.PowersortError):
        binding.set_tuning({"merge_levels": 3})
    assert binding.get_tuning()["merge_levels"] == 1
    binding.set_tuning({"merge_levels": 2})
    assert binding.get_tuning()["merge_levels"] == 2
    binding.set_tuning(None)
    assert binding.get_tuning() == d


def test_no_alloc_entry_point_rejects_before_launch(lib):
    """ps_sort_no_alloc checks its limit and options before touching a device."""
    from paper_1805_04154_amd import binding
    fake = ctypes.c_void_p(0x1000)
    cap = 128 << 20

    def largest(kt, hp):
        # largest n whose scratch fits the fixed 128 MiB array
        lo, hi = 1, 1 << 31
        while lo < hi:
            m = (lo + hi + 1) // 2
            if lib.ps_workspace_bytes(m, 1, kt, hp, None) <= cap:
                lo = m
            else:
                hi = m - 1
        return lo

    # the limits the header states (int32 / int64 keys, with and without payload)
    text = " ".join(re.sub(r"^\s*\*", "", line) for line in open(HEADER).read().splitlines())
    text = " ".join(text.split())
    m = re.search(r"above ([\d ]+) 4-byte keys with a payload \(([\d ]+) without\) or ([\d ]+) 8-byte keys "
                  r"with a payload \(([\d ]+) without\)", text)
    stated = [int(g.replace(" ", "")) for g in m.groups()]
    assert stated == [largest(0, 1), largest(0, 0), largest(2, 1), largest(2, 0)]
    lo = stated[0]
    assert lib.ps_sort_no_alloc(fake, fake, lo + 1, 0, None, None, None) == -2
    assert b"fixed scratch" in lib.ps_last_error()
    assert lib.ps_sort_no_alloc(fake, None, 1 << 31, 0, None, None, None) == -2
    o = binding.PsOptions(ctypes.sizeof(binding.PsOptions), 0, 0, 0, 0x2000, 1 << 30)
    assert lib.ps_sort_no_alloc(fake, fake, 100, 0, ctypes.byref(o), None, None) == -1
    assert b"workspace" in lib.ps_last_error()
    assert lib.ps_sort_no_alloc(fake, None, 10, 0, _opts(binding, min_run=65), None, None) == -5
    assert lib.ps_sort_no_alloc(None, None, 10, 0, None, None, None) == -1


def test_binding_rejects_mismatched_tensors():
    """The binding checks sizes and dtypes of every array the library would
    index before anything reaches the device."""
    import torch
    from paper_1805_04154_amd import binding
    k = torch.zeros(10, dtype=torch.int32)
    off = torch.tensor([0, 4, 10], dtype=torch.int64)
    pay_short = torch.zeros(9, dtype=torch.int32)
    with pytest.raises(ValueError, match="payload"):
        binding.segmented_sort(k, pay_short, off)
    with pytest.raises(ValueError, match="payload"):
        binding.segmented_sort(k, torch.zeros(10, dtype=torch.int64), off)
    with pytest.raises(ValueError, match="payload"):
        binding.sort(k, pay_short)
    with pytest.raises(ValueError, match="payload"):
        binding.sort_no_alloc(k, pay_short)
    with pytest.raises(ValueError, match="offsets"):
        binding.segmented_sort(k, None, off.to(torch.int32))
    with pytest.raises(ValueError, match="offsets"):
        binding.segmented_sort(k, None, torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="offsets"):
        binding.segmented_sort(k, None, off.view(1, 3))
    with pytest.raises(ValueError, match="merge_costs"):
        binding.segmented_sort(k, None, off, merge_costs=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="merge_costs"):
        binding.segmented_sort(k, None, off, merge_costs=torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError, match="status"):
        binding.segmented_sort(k, None, off, status=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="status"):
        binding.segmented_sort(k, None, off, status=torch.zeros(0, dtype=torch.int32))
    with pytest.raises(ValueError, match="merge_cost"):
        binding.sort(k, None, merge_cost=torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError, match="out"):
        binding.merge_cost(k, out=torch.zeros(0, dtype=torch.int64))
    with pytest.raises(ValueError, match="out"):
        binding.segmented_merge_cost(k, off, out=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="status"):
        binding.segmented_merge_cost(k, off, status=torch.zeros(1, dtype=torch.float32))
    with pytest.raises(ValueError, match="offsets"):
        binding.inspect(k, offsets=off.to(torch.int32))
    # well-formed host tensors get as far as the device check
    with pytest.raises(ValueError, match="GPU"):
        binding.segmented_sort(k, torch.zeros(10, dtype=torch.int32), off,
                               merge_costs=torch.zeros(2, dtype=torch.int64),
                               status=torch.zeros(1, dtype=torch.int32))


def test_pool_limit_reports_out_of_memory_before_launch(lib):
    """A call whose scratch exceeds the pool limit fails with
    PS_ERR_OUT_OF_MEMORY before touching a device or enqueuing anything."""
    fake = ctypes.c_void_p(0x1000)
    need = lib.ps_workspace_bytes(1 << 20, 1, 0, 1, None)
    try:
        assert lib.ps_set_pool_limit(need - 1) == 0
        assert lib.ps_sort(fake, fake, 1 << 20, 0, None, None, None) == -3
        assert b"pool limit" in lib.ps_last_error()
        off = ctypes.c_void_p(0x2000)
        assert lib.ps_segmented_sort(fake, fake, off, 3, 1 << 20, 0, None, None, None, None) == -3
        assert lib.ps_merge_cost(fake, 1 << 26, 0, None, fake, None) == -3  # metadata alone
    finally:
        lib.ps_set_pool_limit(0)
