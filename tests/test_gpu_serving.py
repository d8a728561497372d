"""Serving loop: every request's result equals the oracle's, the same whether
it is served alone or batched with others, under a tight HBM budget too."""
import numpy as np
import pytest

from paper_1805_04154_amd import workloads as W

pytestmark = pytest.mark.gpu


def make_requests(metas, keys, torch):
    from paper_1805_04154_amd import batched, serving
    reqs = []
    for i, (m, k) in enumerate(zip(metas, keys)):
        reqs.append(serving.ServedRequest(i, m.arrival_s, batched.to_device(k),
                                          batched.to_device(W.payload_for(m.n))))
    return reqs


def make_pool_requests(metas, keys, torch):
    """The same requests with buffers from one RequestPool per key type."""
    from paper_1805_04154_amd import serving
    need = {}
    for k in keys:
        dt = torch.from_numpy(k[:0]).dtype
        need[dt] = need.get(dt, 0) + len(k)
    pools = {dt: serving.RequestPool(dt, n) for dt, n in need.items()}
    reqs = []
    for i, (m, k) in enumerate(zip(metas, keys)):
        r = pools[torch.from_numpy(k[:0]).dtype].request(i, m.arrival_s, m.n)
        r.keys.copy_(torch.from_numpy(k))
        r.payload.copy_(torch.from_numpy(W.payload_for(m.n).view(np.int32)).view(torch.uint32))
        reqs.append(r)
    torch.cuda.synchronize()
    return reqs


def host(t, dtype):
    import torch
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    return t.cpu().numpy().view(dtype)


@pytest.fixture(scope="module")
def trace():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    metas = W.trace_meta(rate_hz=4000, duration_s=0.03, lo_exp=6, hi_exp=16, seed_index=11)
    keys = W.materialize(metas, workers=1)
    import oracle
    refs = [oracle.powersort(k, W.payload_for(len(k))) for k in keys]
    return metas, keys, refs


def check(done, refs, keys):
    assert len(done) == len(refs)
    for r in done:
        ref = refs[r.rid]
        assert np.array_equal(host(r.keys, keys[r.rid].dtype).view(np.uint8), ref.keys.view(np.uint8)), r.rid
        assert np.array_equal(host(r.payload, np.uint32), ref.payload), r.rid
        assert r.merge_cost == ref.merge_cost, r.rid


def test_batched_serving_matches_oracle(trace):
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    assert len({k.dtype for k in keys}) == 3
    reqs = make_requests(metas, keys, torch)
    srv = serving.SortServer(hbm_budget_bytes=1 << 30, slots=2)
    done = srv.serve(reqs)
    torch.cuda.synchronize()
    check(done, refs, keys)
    st = serving.latency_stats(done)
    assert st["p50_ms"] <= st["p99_ms"]


def test_alone_equals_in_the_mix(trace):
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    mixed = make_requests(metas, keys, torch)
    serving.SortServer(hbm_budget_bytes=1 << 30, slots=3).serve(mixed, realtime=False)
    torch.cuda.synchronize()
    for i in range(0, len(metas), max(1, len(metas) // 12)):
        alone = make_requests([metas[i]], [keys[i]], torch)
        alone[0].rid = 0
        serving.SortServer(hbm_budget_bytes=1 << 28, slots=1).serve(alone, realtime=False)
        torch.cuda.synchronize()
        m = next(r for r in mixed if r.rid == i)
        assert torch.equal(alone[0].keys.view(torch.uint8) if alone[0].keys.dtype != torch.uint8 else alone[0].keys,
                           m.keys.view(torch.uint8)), i
        assert torch.equal(alone[0].payload.view(torch.int32), m.payload.view(torch.int32)), i
        assert alone[0].merge_cost == m.merge_cost == refs[i].merge_cost


def test_tight_budget_and_plain(trace):
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    biggest = max(m.n for m in metas)
    reqs = make_requests(metas, keys, torch)
    # room for one or two requests at a time: admission waits for memory
    srv = serving.SortServer(hbm_budget_bytes=2 * serving.batch_bytes(biggest, 1, torch.int64, False) + (1 << 20),
                             slots=2)
    done = srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)
    reqs = make_requests(metas, keys, torch)
    done = serving.serve_plain(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)


def test_oversized_request_is_rejected(trace):
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    big = max(range(len(metas)), key=lambda i: metas[i].n)
    reqs = make_requests([metas[big]], [keys[big]], torch)
    srv = serving.SortServer(hbm_budget_bytes=serving.batch_bytes(metas[big].n // 2, 1, torch.int32, True), slots=1)
    with pytest.raises(ValueError):
        srv.serve(reqs, realtime=False)


def test_pool_requests_sorted_in_place(trace):
    # requests from pools are batched as slices of them and sorted there;
    # under a tight budget the batches break at different places
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    biggest = max(m.n for m in metas)
    tight = 2 * serving.batch_bytes(biggest, 1, torch.int64, True) + (1 << 20)
    for budget, slots in ((1 << 30, 2), (tight, 2), (1 << 30, 1)):
        reqs = make_pool_requests(metas, keys, torch)
        done = serving.SortServer(hbm_budget_bytes=budget, slots=slots).serve(reqs, realtime=False)
        torch.cuda.synchronize()
        check(done, refs, keys)
    reqs = make_pool_requests(metas, keys, torch)
    done = serving.serve_plain(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)


def test_pool_and_plain_requests_mixed(trace):
    # every third request has buffers of its own: pool batches stop at it
    import torch
    from paper_1805_04154_amd import serving
    metas, keys, refs = trace
    pooled = make_pool_requests(metas, keys, torch)
    own = make_requests(metas, keys, torch)
    reqs = [own[i] if i % 3 == 0 else pooled[i] for i in range(len(metas))]
    done = serving.SortServer(hbm_budget_bytes=1 << 30, slots=2).serve(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)


def test_admission_waits_for_memory_with_a_slot_idle():
    """Four equal requests, each needing B bytes of arena, under a budget of
    1.5 B and two slots: only one batch fits at a time, so the second slot
    stays idle while the first holds the memory, and every result is still
    the oracle's."""
    import torch
    import oracle
    from paper_1805_04154_amd import batched, serving
    n = 1 << 16
    rng = W.make_rng(77)
    keys = [W.random_runs(rng, n, 256.0, 0.25).astype(np.int32) for _ in range(4)]
    refs = [oracle.powersort(k, W.payload_for(n)) for k in keys]
    reqs = [serving.ServedRequest(i, 0.0, batched.to_device(k), batched.to_device(W.payload_for(n)))
            for i, k in enumerate(keys)]
    one = serving.batch_bytes(n, 1, torch.int32, False)
    assert serving.batch_bytes(2 * n, 2, torch.int32, False) > one * 3 // 2
    srv = serving.SortServer(hbm_budget_bytes=one * 3 // 2, slots=2)
    done = srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)
    assert srv.stats["batches"] == 4
    assert srv.stats["max_inflight"] == 1
    assert srv.stats["memory_waits"] > 0
    assert srv.stats["peak_bytes"] <= srv.budget
    # with room for two, both slots are used
    srv2 = serving.SortServer(hbm_budget_bytes=2 * one + (1 << 20), slots=2, max_batch_keys=n)
    reqs = [serving.ServedRequest(i, 0.0, batched.to_device(k), batched.to_device(W.payload_for(n)))
            for i, k in enumerate(keys)]
    done = srv2.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)
    assert srv2.stats["max_inflight"] == 2


def real_size_trace():
    """Thirty requests at the served workload's real sizes (log-uniform in
    [2^12, 2^24]) and key types, with an int64 request of 2^24 keys, a
    float32 request above 2^22 and an int64 request above 2^22 forced in."""
    metas = W.trace_meta(rate_hz=2000, duration_s=1.0, lo_exp=12, hi_exp=24, seed_index=21, max_requests=30)
    forced = {3: (1 << 24, np.int64), 11: ((1 << 22) + 4097, np.float32), 19: ((1 << 22) + 123, np.int64),
              25: ((1 << 23) - 5, np.int32)}
    for i, (n, dt) in forced.items():
        metas[i].n, metas[i].dtype = n, np.dtype(dt)
    return metas


def test_real_size_requests_alone_and_in_the_mix():
    import concurrent.futures as cf
    import torch
    import oracle
    from paper_1805_04154_amd import serving
    metas = real_size_trace()
    print(f"serving parity at real sizes: {len(metas)} requests, {sum(m.n for m in metas)} keys", flush=True)
    keys = W.materialize(metas, workers=1)
    assert {k.dtype for k in keys} == {np.dtype(np.int32), np.dtype(np.int64), np.dtype(np.float32)}
    assert max(m.n for m in metas) == 1 << 24
    with cf.ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda k: oracle.powersort(k, W.payload_for(len(k)), details=False), keys))
    # in the mix: pool requests sorted in place and gathered requests, two slots
    pooled = make_pool_requests(metas, keys, torch)
    own = make_requests(metas, keys, torch)
    mixed = [own[i] if i % 4 == 0 else pooled[i] for i in range(len(metas))]
    srv = serving.SortServer(hbm_budget_bytes=8 << 30, slots=2)
    done = srv.serve(mixed, realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)
    assert srv.stats["batches"] < len(metas)  # requests were batched
    # alone: one request per server call
    for i in range(len(metas)):
        alone = make_requests([metas[i]], [keys[i]], torch)
        alone[0].rid = 0
        serving.SortServer(hbm_budget_bytes=2 << 30, slots=1).serve(alone, realtime=False)
        torch.cuda.synchronize()
        check(alone, [refs[i]], [keys[i]])
    # the plain per-request path too
    done = serving.serve_plain(make_requests(metas, keys, torch), realtime=False)
    torch.cuda.synchronize()
    check(done, refs, keys)
