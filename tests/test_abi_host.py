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
    assert lib.ps_segmented_sort(fake, None, fake, 2, 1 << 32, 0, None, None, None, None) == -2
    # u32 positions: n_total itself must stay below 2^31
    assert lib.ps_segmented_sort(fake, None, fake, 2, 1 << 31, 0, None, None, None, None) == -2
    assert b"2^31" in lib.ps_last_error()
    assert lib.ps_segmented_merge_cost(fake, fake, 2, 1 << 31, 0, None, fake, None, None) == -2
    assert lib.ps_workspace_bytes(1 << 31, 2, 0, 1, None) == 0
    assert lib.ps_workspace_bytes((1 << 31) - 1, 2, 0, 1, None) > 0
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
    # scratch for two copies of keys+payload plus metadata well below the data size
    assert 2 * (1 << 28) * 8 <= big < 2 * (1 << 28) * 8 * 1.25
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
    binding.set_tuning(None)
    assert binding.get_tuning() == d
