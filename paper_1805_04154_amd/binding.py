"""Thin ctypes binding of the powersort HIP library (include/powersort_hip.h).

Only argument marshalling happens here: torch tensors provide device memory
and the current HIP stream; every step of the method runs in the library's
kernels.  There is no fallback: if the library is missing or a call fails,
an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# The in-tree build; POWERSORT_HIP_LIB may name another build of the same
# library (e.g. one with host-side sanitizers for the ABI checks).
LIB_PATH = os.environ.get("POWERSORT_HIP_LIB") or os.path.join(_HERE, "libpowersort_hip.so")

PS_OK = 0
STATUS_NAMES = {0: "PS_OK", -1: "PS_ERR_INVALID_ARG", -2: "PS_ERR_TOO_LARGE", -3: "PS_ERR_OUT_OF_MEMORY",
                -4: "PS_ERR_HIP", -5: "PS_ERR_UNSUPPORTED"}
KEY_TYPES = {torch.int32: 0, torch.uint32: 1, torch.int64: 2, torch.uint64: 3, torch.float32: 4}

# Every symbol include/powersort_hip.h declares.
EXPORTS = ("ps_workspace_bytes", "ps_sort", "ps_sort_no_alloc", "ps_segmented_sort", "ps_merge_cost",
           "ps_segmented_merge_cost",
           "ps_inspect", "ps_alphabetic_tree", "ps_set_tuning", "ps_get_tuning", "ps_profile_enable",
           "ps_profile_read", "ps_set_pool_limit", "ps_release",
           "ps_status_string", "ps_last_error")
TUNING_FIELDS = ("grid_big_leaf", "grid_fused", "grid_merge", "grid_split", "merge_tile", "merge_levels")
PROF_GROUPS = ("partition", "tree", "lists", "big_leaf", "fused", "merge", "split")


class PsOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("min_run", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64)]


class PsInspectOut(ctypes.Structure):
    _fields_ = [("starts", ctypes.c_void_p), ("powers", ctypes.c_void_p), ("node_left", ctypes.c_void_p),
                ("node_right", ctypes.c_void_p), ("leaf_depth", ctypes.c_void_p), ("r", ctypes.c_void_p)]


class PsTuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32)] + [(f, ctypes.c_uint32) for f in TUNING_FIELDS]


class PsProfile(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("calls", ctypes.c_uint32),
                ("launches", ctypes.c_uint32 * 7), ("ms", ctypes.c_double * 7), ("elems", ctypes.c_uint64 * 7)]


class PowersortError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpowersort_hip.so (built by paper_1805_04154_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1805_04154_amd.build` "
                          "(the sort has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    opt = ctypes.POINTER(PsOptions)
    lib.ps_workspace_bytes.restype = ctypes.c_size_t
    lib.ps_workspace_bytes.argtypes = [u64, u64, i32, i32, opt]
    lib.ps_sort.restype = i32
    lib.ps_sort.argtypes = [vp, vp, u64, i32, opt, vp, vp]
    lib.ps_sort_no_alloc.restype = i32
    lib.ps_sort_no_alloc.argtypes = [vp, vp, u64, i32, opt, vp, vp]
    lib.ps_segmented_sort.restype = i32
    lib.ps_segmented_sort.argtypes = [vp, vp, vp, u64, u64, i32, opt, vp, vp, vp]
    lib.ps_merge_cost.restype = i32
    lib.ps_merge_cost.argtypes = [vp, u64, i32, opt, vp, vp]
    lib.ps_segmented_merge_cost.restype = i32
    lib.ps_segmented_merge_cost.argtypes = [vp, vp, u64, u64, i32, opt, vp, vp, vp]
    lib.ps_inspect.restype = i32
    lib.ps_inspect.argtypes = [vp, vp, u64, u64, i32, opt, ctypes.POINTER(PsInspectOut), vp]
    lib.ps_alphabetic_tree.restype = i32
    lib.ps_alphabetic_tree.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp, vp]
    lib.ps_set_tuning.restype = i32
    lib.ps_set_tuning.argtypes = [ctypes.POINTER(PsTuning)]
    lib.ps_get_tuning.restype = i32
    lib.ps_get_tuning.argtypes = [ctypes.POINTER(PsTuning)]
    lib.ps_profile_enable.restype = i32
    lib.ps_profile_enable.argtypes = [i32]
    lib.ps_profile_read.restype = i32
    lib.ps_profile_read.argtypes = [ctypes.POINTER(PsProfile), i32]
    lib.ps_set_pool_limit.restype = i32
    lib.ps_set_pool_limit.argtypes = [u64]
    lib.ps_release.restype = i32
    lib.ps_release.argtypes = [vp]
    lib.ps_status_string.restype = ctypes.c_char_p
    lib.ps_status_string.argtypes = [i32]
    lib.ps_last_error.restype = ctypes.c_char_p
    lib.ps_last_error.argtypes = []
    _ = u32
    _lib = lib
    return lib


def _check(status: int):
    if status != PS_OK:
        msg = _lib.ps_last_error().decode()
        raise PowersortError(status, msg)


METHODS = {"powersort": 0, "peeksort": 1}  # ps_options.flags (PS_FLAG_PEEKSORT = 1)
FLAG_COMPACT_SCRATCH = 2  # PS_FLAG_COMPACT_SCRATCH


def _opts(min_run: int | None, workspace: torch.Tensor | None = None, method: str = "powersort",
          compact_scratch: bool = False):
    if method not in METHODS:
        raise ValueError(f"method must be one of {sorted(METHODS)}")
    if min_run is None and workspace is None and method == "powersort" and not compact_scratch:
        return None
    flags = METHODS[method] | (FLAG_COMPACT_SCRATCH if compact_scratch else 0)
    o = PsOptions(ctypes.sizeof(PsOptions), int(min_run or 0), flags, 0, None, 0)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return ctypes.byref(o)


def _key_type(t: torch.Tensor) -> int:
    if t.dtype not in KEY_TYPES:
        raise TypeError(f"unsupported key dtype {t.dtype}")
    return KEY_TYPES[t.dtype]


def _dev_check(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _check_payload(keys: torch.Tensor, payload: torch.Tensor | None):
    if payload is not None and (payload.dtype not in (torch.int32, torch.uint32) or payload.numel() != keys.numel()):
        raise ValueError("payload must be a 32-bit tensor with one entry per key")


def _check_words(t: torch.Tensor | None, name: str, dtypes: tuple, count: int):
    """t (if given) must hold at least count elements of one of dtypes."""
    if t is None:
        return
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    if t.numel() < count:
        raise ValueError(f"{name} needs at least {count} elements, has {t.numel()}")


_U64 = (torch.int64, torch.uint64)
_I32 = (torch.int32,)


def _check_offsets(offsets: torch.Tensor) -> int:
    """Segment offsets: a 1-D 64-bit tensor of num_segments + 1 >= 2 entries; returns num_segments."""
    if offsets.dtype not in _U64 or offsets.dim() != 1 or offsets.numel() < 2:
        raise ValueError("offsets must be a 1-D int64 tensor of num_segments + 1 >= 2 entries")
    return offsets.numel() - 1


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def workspace_bytes(n_total: int, num_segments: int, dtype: torch.dtype, has_payload: bool,
                    min_run: int | None = None, method: str = "powersort", compact_scratch: bool = False) -> int:
    lib = load_library()
    return int(lib.ps_workspace_bytes(n_total, num_segments, KEY_TYPES[dtype], int(has_payload),
                                      _opts(min_run, None, method, compact_scratch)))


def sort(keys: torch.Tensor, payload: torch.Tensor | None = None, min_run: int | None = None,
         merge_cost: torch.Tensor | None = None, stream=None, workspace: torch.Tensor | None = None,
         method: str = "powersort", compact_scratch: bool = False):
    """Stable in-place powersort (or peeksort) of a 1-D device tensor (payload permuted alongside).

    merge_cost: optional 1-element int64 device tensor that receives M (as uint64 bits)."""
    lib = load_library()
    _check_payload(keys, payload)
    _check_words(merge_cost, "merge_cost", _U64, 1)
    _dev_check(keys, payload, merge_cost)
    _check(lib.ps_sort(keys.data_ptr(), payload.data_ptr() if payload is not None else None, keys.numel(),
                       _key_type(keys), _opts(min_run, workspace, method, compact_scratch),
                       merge_cost.data_ptr() if merge_cost is not None else None, _stream(stream)))
    return keys, payload


def sort_no_alloc(keys: torch.Tensor, payload: torch.Tensor | None = None, min_run: int | None = None,
                  merge_cost: torch.Tensor | None = None, stream=None, method: str = "powersort",
                  compact_scratch: bool = False):
    """sort() in the library's fixed device scratch (ps_sort_no_alloc): no
    device allocation, for inputs whose scratch fits 128 MiB.  Calls that
    overlap on one device race: serialise them (e.g. on one stream)."""
    lib = load_library()
    _check_payload(keys, payload)
    _check_words(merge_cost, "merge_cost", _U64, 1)
    _dev_check(keys, payload, merge_cost)
    _check(lib.ps_sort_no_alloc(keys.data_ptr(), payload.data_ptr() if payload is not None else None, keys.numel(),
                                _key_type(keys), _opts(min_run, None, method, compact_scratch),
                                merge_cost.data_ptr() if merge_cost is not None else None, _stream(stream)))
    return keys, payload


def segmented_sort(keys: torch.Tensor, payload: torch.Tensor | None, offsets: torch.Tensor,
                   min_run: int | None = None, merge_costs: torch.Tensor | None = None,
                   status: torch.Tensor | None = None, stream=None, workspace: torch.Tensor | None = None,
                   method: str = "powersort", compact_scratch: bool = False):
    """Sort every segment [offsets[g], offsets[g+1]) independently (offsets: int64 device tensor)."""
    lib = load_library()
    _check_payload(keys, payload)
    nseg = _check_offsets(offsets)
    _check_words(merge_costs, "merge_costs", _U64, nseg)
    _check_words(status, "status", _I32, 1)
    _dev_check(keys, payload, offsets, merge_costs, status)
    _check(lib.ps_segmented_sort(keys.data_ptr(), payload.data_ptr() if payload is not None else None,
                                 offsets.data_ptr(), nseg, keys.numel(), _key_type(keys),
                                 _opts(min_run, workspace, method, compact_scratch),
                                 merge_costs.data_ptr() if merge_costs is not None else None,
                                 status.data_ptr() if status is not None else None, _stream(stream)))
    return keys, payload


def merge_cost(keys: torch.Tensor, min_run: int | None = None, out: torch.Tensor | None = None,
               stream=None, method: str = "powersort") -> torch.Tensor:
    """Merge cost M of powersort (or peeksort) on keys (keys untouched); returns a 1-element int64 device tensor."""
    lib = load_library()
    _check_words(out, "out", _U64, 1)
    _dev_check(keys, out)
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=keys.device)
    _check(lib.ps_merge_cost(keys.data_ptr(), keys.numel(), _key_type(keys), _opts(min_run, None, method),
                             out.data_ptr(),
                             _stream(stream)))
    return out


def segmented_merge_cost(keys: torch.Tensor, offsets: torch.Tensor, min_run: int | None = None,
                         out: torch.Tensor | None = None, status: torch.Tensor | None = None,
                         stream=None, method: str = "powersort") -> torch.Tensor:
    lib = load_library()
    nseg = _check_offsets(offsets)
    _check_words(out, "out", _U64, nseg)
    _check_words(status, "status", _I32, 1)
    _dev_check(keys, offsets, out, status)
    if out is None:
        out = torch.empty(nseg, dtype=torch.int64, device=keys.device)
    _check(lib.ps_segmented_merge_cost(keys.data_ptr(), offsets.data_ptr(), nseg, keys.numel(), _key_type(keys),
                                       _opts(min_run, None, method), out.data_ptr(),
                                       status.data_ptr() if status is not None else None, _stream(stream)))
    return out


def inspect(keys: torch.Tensor, offsets: torch.Tensor | None = None, min_run: int | None = None,
            stream=None, method: str = "powersort") -> dict:
    """Leaf starts, powers (peeksort: node depth + 1), node leaf ranges and leaf depths
    (as device tensors, trimmed to r)."""
    lib = load_library()
    if offsets is not None:
        _check_offsets(offsets)
    _dev_check(keys, offsets)
    n = keys.numel()
    dev = keys.device
    starts = torch.zeros(n + 1, dtype=torch.int32, device=dev)
    powers = torch.zeros(n + 1, dtype=torch.uint8, device=dev)
    left = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    right = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    depth = torch.zeros(max(n, 1), dtype=torch.uint8, device=dev)
    r = torch.zeros(1, dtype=torch.int32, device=dev)
    out = PsInspectOut(starts.data_ptr(), powers.data_ptr(), left.data_ptr(), right.data_ptr(), depth.data_ptr(),
                       r.data_ptr())
    nseg = 1 if offsets is None else offsets.numel() - 1
    _check(lib.ps_inspect(keys.data_ptr(), offsets.data_ptr() if offsets is not None else None, nseg, n,
                          _key_type(keys), _opts(min_run, None, method), ctypes.byref(out), _stream(stream)))
    rr = int(r.item())
    return {"r": rr, "starts": starts[: rr + 1], "powers": powers[: rr + 1], "node_left": left[:rr],
            "node_right": right[:rr], "leaf_depth": depth[:rr]}


def alphabetic_tree(weights: torch.Tensor, stream=None) -> dict:
    """Method 2' nearly-optimal alphabetic tree for integer leaf weights (a 1-D
    int32/uint32 device tensor, every weight >= 1, sum < 2^31): node powers,
    node leaf ranges, leaf depths, the weighted path length and a status word
    (device tensors)."""
    lib = load_library()
    _dev_check(weights)
    if weights.dtype not in (torch.int32, torch.uint32):
        raise TypeError("weights must be a 32-bit integer tensor")
    r = weights.numel()
    dev = weights.device
    powers = torch.zeros(r + 1, dtype=torch.uint8, device=dev)
    left = torch.zeros(max(r, 1), dtype=torch.int32, device=dev)
    right = torch.zeros(max(r, 1), dtype=torch.int32, device=dev)
    depth = torch.zeros(max(r, 1), dtype=torch.uint8, device=dev)
    cost = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.full((1,), 99, dtype=torch.int32, device=dev)
    _check(lib.ps_alphabetic_tree(weights.data_ptr(), r, powers.data_ptr(), left.data_ptr(), right.data_ptr(),
                                  depth.data_ptr(), cost.data_ptr(), status.data_ptr(), _stream(stream)))
    return {"powers": powers, "node_left": left[:r], "node_right": right[:r], "leaf_depth": depth[:r],
            "cost": cost, "status": status}


def set_tuning(tuning: dict | None):
    """Set the launch shape (dict with any of TUNING_FIELDS; None = defaults)."""
    lib = load_library()
    if tuning is None:
        _check(lib.ps_set_tuning(None))
        return
    t = PsTuning()
    t.struct_size = ctypes.sizeof(PsTuning)
    for f in TUNING_FIELDS:
        setattr(t, f, int(tuning.get(f, 0)))
    _check(lib.ps_set_tuning(ctypes.byref(t)))


def get_tuning() -> dict:
    lib = load_library()
    t = PsTuning()
    t.struct_size = ctypes.sizeof(PsTuning)
    _check(lib.ps_get_tuning(ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def profile_enable(on: bool = True, groups=None):
    """Time the library's kernel groups with HIP events on the caller's stream:
    every group, or only the named ones (e.g. ``groups=("merge",)``)."""
    lib = load_library()
    if not on:
        mask = 0
    elif groups is None:
        mask = 1
    else:
        mask = 0
        for g in groups:
            mask |= 1 << PROF_GROUPS.index(g)
        if mask == 1:
            raise ValueError("timing the partition group alone is not expressible; add another group")
    _check(lib.ps_profile_enable(mask))


def profile_read(reset: bool = False) -> dict:
    """Accumulated per-group {launches, ms, elems} since the last reset."""
    lib = load_library()
    p = PsProfile()
    p.struct_size = ctypes.sizeof(PsProfile)
    _check(lib.ps_profile_read(ctypes.byref(p), int(reset)))
    return {"calls": p.calls,
            **{g: {"launches": p.launches[i], "ms": p.ms[i], "elems": p.elems[i]} for i, g in enumerate(PROF_GROUPS)}}


def set_pool_limit(nbytes: int):
    """Cap the library's per-stream scratch (0 = no cap): larger calls fail
    with PS_ERR_OUT_OF_MEMORY before anything is enqueued."""
    _check(load_library().ps_set_pool_limit(int(nbytes)))


def release(stream=None):
    lib = load_library()
    _check(lib.ps_release(_stream(stream)))
