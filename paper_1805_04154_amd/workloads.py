"""Seeded synthetic inputs shaped like the workloads of the powersort study.

This module only draws random data; it holds none of the sorting method's
arithmetic and is shared by the GPU tests, the oracle tests and the benchmark
so that both sides see the same bytes.

Input families:
  * random permutations and the "random-runs" model of Sec. 4.1 (a random
    permutation whose segments, of geometric lengths with mean l, are sorted;
    here a fraction of the segments is reversed, which makes them strictly
    descending because permutation values are distinct);
  * concatenated ascending / strictly descending runs with uniform or Zipf
    run lengths and iid keys from a bounded range (duplicates exercise
    stability);
  * segmented batches with log-uniform sizes and a Poisson request trace.

Every generator takes an explicit ``numpy.random.Generator`` or seed.
Payloads are the original indices (``arange(n, dtype=uint32)``).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

BASE_SEED = 1805_04154


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def config_rng(index: int) -> np.random.Generator:
    """Generator for workload number ``index`` (0-based) of the fixed set below."""
    return make_rng(BASE_SEED + index)


# ---------------------------------------------------------------- run building


def _sorted_iid(rng: np.random.Generator, length: int, lo: int, hi: int) -> np.ndarray:
    """``length`` iid uniform integers from [lo, hi), returned in ascending order.

    Uses the order statistics of uniforms (normalised partial sums of
    exponential gaps), which is O(length) and has the same distribution as
    sorting iid draws."""
    if length == 0:
        return np.zeros(0, np.int64)
    gaps = rng.exponential(size=length + 1)
    c = np.cumsum(gaps)
    u = c[:-1] / c[-1]
    v = lo + np.floor(u * (hi - lo)).astype(np.int64)
    return np.minimum(v, hi - 1)


def _distinct_desc(rng: np.random.Generator, length: int, lo: int, hi: int) -> np.ndarray:
    """``length`` distinct integers from [lo, hi) in strictly descending order."""
    span = hi - lo
    if length > span:
        raise ValueError("cannot draw that many distinct values")
    if span <= (1 << 22):
        v = lo + rng.choice(span, size=length, replace=False).astype(np.int64)
    else:
        got = np.zeros(0, np.int64)
        while got.shape[0] < length:
            more = rng.integers(lo, hi, size=length - got.shape[0] + 16, dtype=np.int64)
            got = np.unique(np.concatenate([got, more]))
        v = rng.permutation(got)[:length]
    return np.sort(v)[::-1].copy()


def concatenated_runs(rng: np.random.Generator, n: int, lengths_fn, key_lo: int, key_hi: int,
                      desc_frac: float, desc_max: int | None = None) -> np.ndarray:
    """Concatenate runs until n keys exist (the last run is clipped).

    ``lengths_fn(rng, k)`` draws k run lengths.  Each run is ascending with iid
    keys from [key_lo, key_hi), or, with probability ``desc_frac``, strictly
    descending with distinct keys (its length clipped to ``desc_max``)."""
    out = np.empty(n, np.int64)
    pos = 0
    while pos < n:
        lens = lengths_fn(rng, 1024)
        desc = rng.random(lens.shape[0]) < desc_frac
        for L, d in zip(lens.tolist(), desc.tolist()):
            if pos >= n:
                break
            if d and desc_max is not None:
                L = min(L, desc_max)
            L = max(1, min(int(L), n - pos))
            if d:
                out[pos:pos + L] = _distinct_desc(rng, L, key_lo, key_hi)
            else:
                out[pos:pos + L] = _sorted_iid(rng, L, key_lo, key_hi)
            pos += L
    return out


def random_runs(rng: np.random.Generator, m: int, mean_len: float, desc_frac: float = 0.0) -> np.ndarray:
    """The random-runs model of Sec. 4.1 on a permutation of 0..m-1.

    Segment lengths are geometric with mean ``mean_len``; each segment holds
    its values in ascending order, and a fraction ``desc_frac`` of segments is
    reversed.  Returns int64 values."""
    if m == 0:
        return np.zeros(0, np.int64)
    p = min(1.0, 1.0 / max(mean_len, 1.0))
    lens = []
    tot = 0
    while tot < m:
        g = rng.geometric(p, size=max(16, int(2 * m / max(mean_len, 1.0)) + 16))
        lens.append(g)
        tot += int(g.sum())
    L = np.concatenate(lens)
    c = np.cumsum(L)
    k = int(np.searchsorted(c, m)) + 1
    L = L[:k].copy()
    L[-1] -= int(c[k - 1] - m)
    # A uniformly random permutation split into blocks of sizes L has block
    # contents distributed as a random arrangement of the multiset of block
    # ids over the values 0..m-1; a stable bucketing of the values by block id
    # lists every block's values in ascending order.
    dt = np.uint16 if k <= 0xFFFF else np.int64
    owner = rng.permutation(np.repeat(np.arange(k, dtype=dt), L))
    vals = np.argsort(owner, kind="stable").astype(np.int64)
    if desc_frac > 0.0:
        rev = rng.random(k) < desc_frac
        starts = np.concatenate([[0], np.cumsum(L)[:-1]])
        idx = np.arange(m, dtype=np.int64)
        blk = np.repeat(np.arange(k), L)
        s = starts[blk]
        e = s + L[blk]
        flip = rev[blk]
        idx[flip] = (s + e - 1 - idx)[flip]
        vals = vals[idx]
    return vals


def random_permutation(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.permutation(n).astype(np.int64)


def payload_for(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint32)


# --------------------------------------------------------------- fixed configs

@dataclass
class Workload:
    name: str
    keys: np.ndarray
    payload: np.ndarray
    offsets: np.ndarray | None = None  # segment offsets (uint64) for batched inputs

    @property
    def n(self) -> int:
        return int(self.keys.shape[0])


def runs_2p20(n: int = 1 << 20, seed_index: int = 0) -> Workload:
    """One array of int32 keys: runs of lengths uniform in [1, 2048], keys uniform
    in [0, 2^16), 25% of runs strictly descending."""
    rng = config_rng(seed_index)
    keys = concatenated_runs(rng, n, lambda r, k: r.integers(1, 2049, size=k), 0, 1 << 16, 0.25)
    return Workload(f"runs_u2048_n{n}_i32", keys.astype(np.int32), payload_for(n))


def permutation_i32(n: int = 1 << 26, seed_index: int = 1) -> Workload:
    """Uniform random permutation of 0..n-1 as int32 keys."""
    rng = config_rng(seed_index)
    return Workload(f"perm_n{n}_i32", random_permutation(rng, n).astype(np.int32), payload_for(n))


def runs_sqrt_i32(n: int = 1 << 26, seed_index: int = 1) -> Workload:
    """Runs of lengths uniform in [1, 2 sqrt(n)], iid keys over the full int32
    range, 25% strictly descending."""
    rng = make_rng(BASE_SEED + 1000 + seed_index)
    hi = 2 * int(math.isqrt(n))
    keys = concatenated_runs(rng, n, lambda r, k: r.integers(1, hi + 1, size=k), -(1 << 31), 1 << 31, 0.25)
    return Workload(f"runs_u{hi}_n{n}_i32", keys.astype(np.int32), payload_for(n))


def zipf_runs(n: int = 1 << 28, key_dtype=np.uint64, seed_index: int = 2) -> Workload:
    """Runs with Zipf(1.2) lengths clipped to [1, 2^24], keys uniform in
    [0, 2^20), 10% strictly descending (descending runs clipped to 2^20, the
    number of distinct keys available)."""
    rng = config_rng(seed_index)
    keys = concatenated_runs(rng, n, lambda r, k: np.minimum(r.zipf(1.2, size=k), 1 << 24),
                             0, 1 << 20, 0.10, desc_max=1 << 20)
    tag = np.dtype(key_dtype).name
    return Workload(f"zipf_runs_n{n}_{tag}", keys.astype(key_dtype), payload_for(n))


def _segment_keys(args):
    """Worker: random-runs keys for one segment, written into shared memory."""
    shm_name, dtype, a, b, seq = args
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        out = np.ndarray((b,), dtype=dtype, buffer=shm.buf)
        m = b - a
        rng = np.random.Generator(np.random.PCG64(seq))
        out[a:b] = random_runs(rng, m, math.sqrt(m), 0.25).astype(dtype)
    finally:
        shm.close()
    return 0


def batched_offsets(nseg: int = 4096, lo_exp: int = 10, hi_exp: int = 22, seed_index: int = 3) -> np.ndarray:
    """Segment offsets of ``batched_random_runs`` (sizes log-uniform in
    [2^lo_exp, 2^hi_exp]) without generating the keys."""
    rng = config_rng(seed_index)
    sizes = np.floor(np.exp(rng.uniform(lo_exp * math.log(2), hi_exp * math.log(2), size=nseg))).astype(np.int64)
    offsets = np.zeros(nseg + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
    return offsets


def batched_random_runs(nseg: int = 4096, lo_exp: int = 10, hi_exp: int = 22, desc_frac: float = 0.25,
                        seed_index: int = 3, key_dtype=np.int32, workers: int | None = None) -> Workload:
    """``nseg`` arrays with sizes log-uniform in [2^lo_exp, 2^hi_exp], each a
    random-runs input with mean run length sqrt(size), 25% of runs reversed.

    Segment g draws from its own generator (spawned from the workload seed),
    so the result does not depend on the number of worker processes."""
    offsets = batched_offsets(nseg, lo_exp, hi_exp, seed_index)
    total = int(offsets[-1])
    seqs = np.random.SeedSequence(BASE_SEED + 100 + seed_index).spawn(nseg)
    dt = np.dtype(key_dtype)
    if desc_frac != 0.25:
        raise ValueError("the batched workload reverses 25% of its runs")
    workers = workers or min(16, os.cpu_count() or 1)
    if total < (1 << 22) or workers <= 1:
        keys = np.empty(total, dt)
        for g in range(nseg):
            a, b = int(offsets[g]), int(offsets[g + 1])
            keys[a:b] = random_runs(np.random.Generator(np.random.PCG64(seqs[g])), b - a,
                                    math.sqrt(b - a), 0.25).astype(dt)
    else:
        import multiprocessing as mp
        from multiprocessing import shared_memory
        shm = shared_memory.SharedMemory(create=True, size=max(1, total * dt.itemsize))
        try:
            jobs = [(shm.name, dt, int(offsets[g]), int(offsets[g + 1]), seqs[g]) for g in range(nseg)]
            jobs.sort(key=lambda j: j[2] - j[3])  # largest first
            with mp.get_context("fork").Pool(workers) as pool:
                for _ in pool.imap_unordered(_segment_keys, jobs, chunksize=4):
                    pass
            keys = np.ndarray((total,), dtype=dt, buffer=shm.buf).copy()
        finally:
            shm.close()
            shm.unlink()
    return Workload(f"batched_{nseg}_logu{lo_exp}-{hi_exp}", keys, payload_for(total), offsets)


def f32_from_values(rng: np.random.Generator, vals: np.ndarray, m: int, specials: bool = True) -> np.ndarray:
    """Map permutation values v to float32 keys v - m/2 (exact below 2^24) and,
    optionally, plant a few signed zeros, infinities and NaNs."""
    f = (vals - m // 2).astype(np.float32)
    if specials and m >= 16:
        pos = rng.choice(m, size=8, replace=False)
        bits = np.array([0x80000000, 0x00000000, 0x7F800000, 0xFF800000,
                         0x7FC00000, 0xFFC00000, 0x7F800001, 0x80000000], np.uint32)
        f[pos] = bits.view(np.float32)
    return f


@dataclass
class Request:
    arrival_s: float
    keys: np.ndarray
    payload: np.ndarray


@dataclass
class RequestMeta:
    arrival_s: float
    n: int
    dtype: np.dtype
    seq: object  # numpy SeedSequence of the request's contents


def trace_meta(rate_hz: float = 2000.0, duration_s: float = 1.0, lo_exp: int = 12, hi_exp: int = 24,
               seed_index: int = 4, max_requests: int | None = None) -> list[RequestMeta]:
    """Open-loop arrivals: exponential inter-arrival times at ``rate_hz``,
    sizes log-uniform in [2^lo_exp, 2^hi_exp], key dtype uniform over
    {int32, int64, float32}; each request carries the seed of its contents."""
    rng = config_rng(seed_index)
    t = 0.0
    out: list[RequestMeta] = []
    kinds = (np.dtype(np.int32), np.dtype(np.int64), np.dtype(np.float32))
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        m = int(math.floor(math.exp(rng.uniform(lo_exp * math.log(2), hi_exp * math.log(2)))))
        out.append(RequestMeta(t, m, kinds[int(rng.integers(0, 3))], None))
    seqs = np.random.SeedSequence(BASE_SEED + 200 + seed_index).spawn(len(out))
    for r, q in zip(out, seqs):
        r.seq = q
    return out


def request_keys(meta: RequestMeta) -> np.ndarray:
    """Contents of one request: random-runs values (mean run length sqrt(n),
    25% reversed) mapped to the request's key type (int64 keys spread over a
    wide range; float32 keys centred on 0 with signed zeros, infinities and
    NaNs planted)."""
    rng = np.random.Generator(np.random.PCG64(meta.seq))
    m = meta.n
    vals = random_runs(rng, m, math.sqrt(m), 0.25)
    if meta.dtype == np.int32:
        return (vals - m // 2).astype(np.int32)
    if meta.dtype == np.int64:
        return (vals - m // 2).astype(np.int64) * np.int64(1 << 20)
    return f32_from_values(rng, vals, m)


def _request_worker(args):
    shm_name, total_bytes, byte_off, meta = args
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        k = request_keys(meta)
        buf = np.ndarray((total_bytes,), dtype=np.uint8, buffer=shm.buf)
        buf[byte_off:byte_off + k.nbytes] = k.view(np.uint8)
    finally:
        shm.close()
    return 0


def materialize(metas: list[RequestMeta], workers: int | None = None) -> list[np.ndarray]:
    """Keys of every request, generated in parallel worker processes."""
    sizes = [m.n * m.dtype.itemsize for m in metas]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(offs[-1])
    workers = workers or min(16, os.cpu_count() or 1)
    if total < (1 << 24) or workers <= 1:
        return [request_keys(m) for m in metas]
    import multiprocessing as mp
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(create=True, size=max(1, total))
    try:
        jobs = [(shm.name, total, int(offs[i]), metas[i]) for i in range(len(metas))]
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_request_worker, jobs, chunksize=2):
                pass
        big = np.ndarray((total,), dtype=np.uint8, buffer=shm.buf).copy()
    finally:
        shm.close()
        shm.unlink()
    return [big[offs[i]:offs[i + 1]].view(metas[i].dtype) for i in range(len(metas))]


def request_trace(rate_hz: float = 2000.0, duration_s: float = 1.0, lo_exp: int = 12, hi_exp: int = 24,
                  seed_index: int = 4, max_requests: int | None = None) -> list[Request]:
    """Requests of trace_meta() with their contents and uint32 payloads."""
    metas = trace_meta(rate_hz, duration_s, lo_exp, hi_exp, seed_index, max_requests)
    keys = materialize(metas)
    return [Request(m.arrival_s, k, payload_for(m.n)) for m, k in zip(metas, keys)]
