"""Powersort oracle -- test infrastructure only.

A thin ctypes wrapper around ``powersort_oracle.c``, a plain single-threaded
CPU powersort written from the definitions of Munro & Wild, "Nearly-Optimal
Mergesorts" (ESA 2018): run convention (Sec. 2), Alg. PowerSort with the
minimum-run extension (Sec. 3.2.2, App. B.3/B.4), Def. "Node Power" evaluated
by its defining loop, stable left-biased merges (App. B.1) and merge cost as
the sum of merge result sizes (Sec. 2.2).

Only ``tests/``, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU path.

Parity status per function (pins live in the tests' oracle-pin suite):
  powersort            pinned: stable-sort output, partition, powers, merge
                       list and merge cost (Fig. 1, entropy bounds, DP optimum,
                       the random-runs merge cost printed in Sec. 4.3)
  segmented_powersort  pinned through powersort (one call per segment)
  merge_order          pinned: Fig. 1 powers/tree/cost, Cartesian tree of the
                       powers, entropy bounds and an interval-DP optimum
  node_power           pinned: Fig. 1 powers and an exact-rational evaluation
  peeksort             pinned: stable-sort output, the same leaves as
                       powersort, Fig. 1's left (Method 1) tree and cost, the
                       bound of Thm. "peeksort", an independent
                       nearest-boundary formulation of the split rule
  segmented_peeksort   pinned through peeksort (one call per segment)
  peek_merge_order     pinned: Fig. 1 left tree, Thm. "peeksort" bound
  topdown_mergesort    pinned: stable-sort output, M = 0 on sorted input, the
  bottomup_mergesort   closed forms of the non-adaptive recursions on strictly
                       decreasing input (no merge check fires), and M
                       recomputed from the original data over the fixed
                       recursion shapes
  Result.comparisons   pinned: exact counts on sorted / reversed / two-run
                       inputs, n - 1 for run detection plus at most size - 1
                       per merge, and the comparison bounds of Thm.
                       "powersort" and "peeksort"
  powersort(galloping=True)
                       pinned: the same output, merges and merge cost as the
                       plain merges and the library stable sort; at least the
                       information bound lg C(a+b, a) per merge; exactly the
                       plain count when the output alternates between runs;
                       logarithmic cost per block when runs supply long
                       blocks
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "powersort_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Key-type numbering of powersort_oracle.c (independent of the product ABI).
KEY_TYPES = {"i32": 0, "u32": 1, "i64": 2, "u64": 3, "f32": 4}
_NP_DTYPE = {"i32": np.int32, "u32": np.uint32, "i64": np.int64, "u64": np.uint64, "f32": np.float32}

DEFAULT_MIN_RUN = 24  # w used in the paper's experiments (App. B.2)


class _Merge(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("mid", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


_SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build_sanitized() -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc) into oracle/liboracle_san.so.  Loading it needs gcc's libasan
    preloaded (see asan_runtime()); select it with ORACLE_LIB."""
    tmp = _SAN_LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", *SANITIZE_FLAGS,
                           "-o", tmp, _SRC])
    os.replace(tmp, _SAN_LIB_PATH)
    return _SAN_LIB_PATH


def asan_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime, for LD_PRELOAD."""
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 into oracle/liboracle.so (or, with
    ORACLE_LIB set in the environment, use that prebuilt library instead)."""
    if os.environ.get("ORACLE_LIB"):
        return os.environ["ORACLE_LIB"]
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_powersort.restype = ctypes.c_int
        lib.oracle_powersort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         u64p, u64p]
        lib.oracle_powersort_galloping.restype = ctypes.c_int
        lib.oracle_powersort_galloping.argtypes = lib.oracle_powersort.argtypes
        lib.oracle_segmented_powersort.restype = ctypes.c_int
        lib.oracle_segmented_powersort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                                   ctypes.c_void_p]
        lib.oracle_merge_order.restype = ctypes.c_int
        lib.oracle_merge_order.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, u64p]
        lib.oracle_node_power.restype = ctypes.c_uint
        lib.oracle_node_power.argtypes = [ctypes.c_uint64] * 5
        lib.oracle_peeksort.restype = ctypes.c_int
        lib.oracle_peeksort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        u64p, u64p]
        lib.oracle_peek_merge_order.restype = ctypes.c_int
        lib.oracle_peek_merge_order.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                ctypes.c_void_p, u64p]
        lib.oracle_last_comparisons.restype = ctypes.c_uint64
        lib.oracle_last_comparisons.argtypes = []
        for name in ("oracle_topdown_mergesort", "oracle_bottomup_mergesort"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, u64p]
        lib.oracle_segmented_peeksort.restype = ctypes.c_int
        lib.oracle_segmented_peeksort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                                  ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def key_type_of(keys: np.ndarray) -> str:
    for name, dt in _NP_DTYPE.items():
        if keys.dtype == dt:
            return name
    raise TypeError(f"unsupported key dtype {keys.dtype}")


class Result:
    """Everything the oracle reports for one powersort call."""

    def __init__(self, keys, payload, starts, powers, merges, merge_cost, depth=None, comparisons=None):
        self.keys = keys            # sorted keys (a new array)
        self.payload = payload      # payload permuted alongside, or None
        self.starts = starts        # uint64[r+1] run starts after min-run extension
        self.powers = powers        # uint8[r-1] boundary powers, left to right (powersort only)
        self.merges = merges        # uint64[r-1, 3] (lo, mid, hi) in execution order
        self.merge_cost = merge_cost
        self.depth = depth          # uint8[r] leaf depths (peeksort only)
        self.comparisons = comparisons  # key comparisons made by the call

    @property
    def r(self) -> int:
        return len(self.starts) - 1


def powersort(keys: np.ndarray, payload: np.ndarray | None = None, min_run: int = DEFAULT_MIN_RUN,
              details: bool = True, galloping: bool = False) -> Result:
    """Run the oracle on copies of keys/payload; inputs are left untouched.
    galloping: merge with Timsort-style galloping (same result and merge
    cost, fewer comparisons when runs supply long blocks)."""
    lib = _load()
    kt = key_type_of(keys)
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    n = k.shape[0]
    r = ctypes.c_uint64(0)
    M = ctypes.c_uint64(0)
    if details:
        starts = np.zeros(n + 1, np.uint64)
        powers = np.zeros(max(n, 1), np.uint8)
        merges = np.zeros((max(n, 1), 3), np.uint64)
    else:
        starts = powers = merges = None
    fn = lib.oracle_powersort_galloping if galloping else lib.oracle_powersort
    rc = fn(_ptr(k), _ptr(p), n, KEY_TYPES[kt], min_run, _ptr(starts), _ptr(powers),
            _ptr(merges), ctypes.byref(r), ctypes.byref(M))
    if rc != 0:
        raise RuntimeError("oracle_powersort failed")
    rr = r.value
    if details:
        starts = starts[: rr + 1].copy()
        powers = powers[: max(rr - 1, 0)].copy()
        merges = merges[: max(rr - 1, 0)].copy()
    return Result(k, p, starts, powers, merges, M.value, comparisons=int(lib.oracle_last_comparisons()))


def segmented_powersort(keys: np.ndarray, payload: np.ndarray | None, offsets: np.ndarray,
                        min_run: int = DEFAULT_MIN_RUN):
    """Sort each segment [offsets[g], offsets[g+1]) independently.

    Returns (sorted keys, permuted payload or None, per-segment merge costs)."""
    lib = _load()
    kt = key_type_of(keys)
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = off.shape[0] - 1
    costs = np.zeros(max(nseg, 1), np.uint64)
    rc = lib.oracle_segmented_powersort(_ptr(k), _ptr(p), _ptr(off), nseg, KEY_TYPES[kt], min_run,
                                        _ptr(costs))
    if rc != 0:
        raise RuntimeError("oracle_segmented_powersort failed")
    return k, p, costs[:nseg].copy()


def merge_order(lengths) -> tuple[np.ndarray, np.ndarray, int]:
    """Alg. PowerSort's merge order for given run lengths (no data moves).

    Returns (powers uint8[r-1], merges uint64[r-1, 3] in execution order, M)."""
    L = np.ascontiguousarray(lengths, dtype=np.uint64)
    r = L.shape[0]
    powers = np.zeros(max(r, 1), np.uint8)
    merges = np.zeros((max(r, 1), 3), np.uint64)
    M = ctypes.c_uint64(0)
    if _load().oracle_merge_order(_ptr(L), r, _ptr(powers), _ptr(merges), ctypes.byref(M)) != 0:
        raise ValueError("run lengths must be positive")
    return powers[: max(r - 1, 0)].copy(), merges[: max(r - 1, 0)].copy(), M.value


def node_power(s1: int, n1: int, s2: int, n2: int, n: int) -> int:
    """Def. "Node Power" for runs [s1, s1+n1) and [s2, s2+n2) of an n-array."""
    return int(_load().oracle_node_power(s1, n1, s2, n2, n))


def peeksort(keys: np.ndarray, payload: np.ndarray | None = None, min_run: int = DEFAULT_MIN_RUN,
             details: bool = True) -> Result:
    """Peeksort (Alg. PeekSort) over the same leaves as powersort, on copies
    of keys/payload.  Merges are reported in post-order; powers is None."""
    lib = _load()
    kt = key_type_of(keys)
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    n = k.shape[0]
    r = ctypes.c_uint64(0)
    M = ctypes.c_uint64(0)
    if details:
        starts = np.zeros(n + 1, np.uint64)
        merges = np.zeros((max(n, 1), 3), np.uint64)
        depth = np.zeros(max(n, 1), np.uint8)
    else:
        starts = merges = depth = None
    rc = lib.oracle_peeksort(_ptr(k), _ptr(p), n, KEY_TYPES[kt], min_run, _ptr(starts), _ptr(merges),
                             _ptr(depth), ctypes.byref(r), ctypes.byref(M))
    if rc != 0:
        raise RuntimeError("oracle_peeksort failed")
    rr = r.value
    if details:
        starts = starts[: rr + 1].copy()
        merges = merges[: max(rr - 1, 0)].copy()
        depth = depth[:rr].copy()
    return Result(k, p, starts, None, merges, M.value, depth, comparisons=int(lib.oracle_last_comparisons()))


def segmented_peeksort(keys: np.ndarray, payload: np.ndarray | None, offsets: np.ndarray,
                       min_run: int = DEFAULT_MIN_RUN):
    """Peeksort of each segment on its own: (keys, payload or None, costs)."""
    lib = _load()
    kt = key_type_of(keys)
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nseg = off.shape[0] - 1
    costs = np.zeros(max(nseg, 1), np.uint64)
    rc = lib.oracle_segmented_peeksort(_ptr(k), _ptr(p), _ptr(off), nseg, KEY_TYPES[kt], min_run, _ptr(costs))
    if rc != 0:
        raise RuntimeError("oracle_segmented_peeksort failed")
    return k, p, costs[:nseg].copy()


def peek_merge_order(lengths) -> tuple[np.ndarray, np.ndarray, int]:
    """Peeksort's merge tree for given run lengths (no data moves).

    Returns (merges uint64[r-1, 3] in post-order, leaf depths uint8[r], M)."""
    L = np.ascontiguousarray(lengths, dtype=np.uint64)
    r = L.shape[0]
    merges = np.zeros((max(r, 1), 3), np.uint64)
    depth = np.zeros(max(r, 1), np.uint8)
    M = ctypes.c_uint64(0)
    if _load().oracle_peek_merge_order(_ptr(L), r, _ptr(merges), _ptr(depth), ctypes.byref(M)) != 0:
        raise ValueError("run lengths must be positive")
    return merges[: max(r - 1, 0)].copy(), depth[:r].copy(), M.value


def _elementary(name: str, keys: np.ndarray, payload: np.ndarray | None, min_run: int) -> Result:
    lib = _load()
    kt = key_type_of(keys)
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    M = ctypes.c_uint64(0)
    if getattr(lib, name)(_ptr(k), _ptr(p), k.shape[0], KEY_TYPES[kt], min_run, ctypes.byref(M)) != 0:
        raise RuntimeError(f"{name} failed")
    return Result(k, p, None, None, None, M.value, comparisons=int(lib.oracle_last_comparisons()))


def topdown_mergesort(keys: np.ndarray, payload: np.ndarray | None = None,
                      min_run: int = DEFAULT_MIN_RUN) -> Result:
    """Top-down mergesort with the already-in-order check before each merge
    and insertion sort below min_run elements (Sec. 4.1), on copies; the
    Result holds keys, payload and merge_cost."""
    return _elementary("oracle_topdown_mergesort", keys, payload, min_run)


def bottomup_mergesort(keys: np.ndarray, payload: np.ndarray | None = None,
                       min_run: int = DEFAULT_MIN_RUN) -> Result:
    """Bottom-up mergesort from insertion-sorted chunks of min_run elements,
    with the already-in-order check before each merge (Sec. 4.1), on copies."""
    return _elementary("oracle_bottomup_mergesort", keys, payload, min_run)
