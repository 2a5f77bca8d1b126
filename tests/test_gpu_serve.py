"""GPU tests of the serving loop: results in the mix equal results alone (exactly --
integer outputs), budgeted admission with eviction, and graph replay vs plain launches."""
import ctypes

import numpy as np
import pytest

from paper_2508_11443_amd import workloads
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2508_11443_amd import fks, serve
    return fks, serve


def small_stream(count, seed):
    return workloads.serving_requests(count, 2000.0, seed, build_lo=1 << 10, build_hi=1 << 16,
                                      lookup_lo=1 << 8, lookup_hi=1 << 14)


def export_handle(fks, handle):
    inf = fks.fks_map_info()
    assert fks.library().fks_info(handle, ctypes.byref(inf)) == 0
    h = np.zeros(inf.header_bytes, np.uint8)
    s = np.zeros(inf.slot_bytes, np.uint8)
    assert fks.library().fks_export(handle, h.ctypes.data if h.size else None,
                                    s.ctypes.data if s.size else None, None) == 0
    return h, s


def test_results_in_the_mix_equal_results_alone():
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    reqs = small_stream(80, 1)
    announce("gpu serve: 80-request mix, closed loop, vs each request alone")
    wl = serve.Workload(reqs, [3000, 20000, 500], 7, dev)
    res, outs = serve.run(wl, 8 << 30, closed_loop=True)
    assert res["status_ok"]
    assert serve.check(wl, outs)
    st = res["stats"]
    assert st["lookup_launches"] >= 1 and st["coalesced_requests"] == res.get("lookup_count", 0)
    # alone: build each target map by itself, run the lookup by itself, compare bit for bit
    alone_maps = {}
    for p, o in zip(wl.plan, outs):
        if p[0] != "lookup":
            continue
        tgt = p[1]
        if tgt not in alone_maps:
            keys, vals, seed, n, _ = wl.maps[tgt]
            alone_maps[tgt] = fks.fks_build_u64(keys, vals, seed)
        q = p[2]
        v = torch.empty(q.numel(), dtype=torch.int32, device=dev)
        f = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
        fks.fks_lookup_u64(alone_maps[tgt], q, v, f)
        torch.cuda.synchronize()
        assert torch.equal(v, o[0]) and torch.equal(f, o[1])


def test_server_maps_equal_standalone_builds():
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: resident map bytes == standalone build")
    srv = fks.FksServer(8 << 30)
    keys = workloads.mix_keys_torch(torch.arange(0, 50000, dtype=torch.int64, device=dev))
    vals = torch.arange(50000, dtype=torch.int32, device=dev)
    _, mid = srv.submit_build(keys, vals, 4242)
    srv.wait_all()
    h1, s1 = export_handle(fks, srv.map_handle(mid))
    alone = fks.fks_build_u64(keys, vals, 4242)
    h2, s2, _ = fks.fks_export(alone)
    assert (h1 == h2).all() and (s1 == s2).all()
    srv.destroy()


def test_budget_admission_and_lru_eviction():
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: budget admission with LRU eviction")
    n = 100000
    per_map = 16 * ((n + 7) // 8) + 16 * 4 * n + 24 * 64 + 4096   # the server's reservation
    # two resident maps (~34 B/key each) plus one reservation exceed 1.7 reservations
    srv = fks.FksServer(int(1.7 * per_map))
    maps = []
    for b in range(3):
        k = workloads.mix_keys_torch(torch.arange(b * n, (b + 1) * n, dtype=torch.int64, device=dev))
        v = torch.arange(n, dtype=torch.int32, device=dev)
        maps.append((k, v))
    _, m0 = srv.submit_build(*maps[0], 1)
    _, m1 = srv.submit_build(*maps[1], 2)
    srv.wait_all()
    # touch map 1 so map 0 is the least recently used
    q1 = maps[1][0][:1000].contiguous()
    v1 = torch.empty(1000, dtype=torch.int32, device=dev)
    f1 = torch.empty(1000, dtype=torch.uint8, device=dev)
    srv.submit_lookup(m1, q1, v1, f1)
    srv.wait_all()
    rid2, m2 = srv.submit_build(*maps[2], 3)
    srv.wait_all()
    assert srv.poll(rid2)[1] == 0
    st = srv.stats()
    assert st["evictions"] >= 1 and st["resident_maps"] <= 2
    assert srv.map_handle(m0) is None or srv.map_handle(m0) == 0
    # a lookup against the evicted map completes with an error status
    rid = srv.submit_lookup(m0, q1, v1, f1)
    srv.wait_all()
    done, status, _ = srv.poll(rid)
    assert done and status != 0
    assert bool(f1.all())   # the earlier lookup on map 1 found its keys
    srv.destroy()


def test_graph_replay_equals_plain_launches():
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: graph replay vs plain launches")
    reqs = small_stream(40, 2)
    wl = serve.Workload(reqs, [4000], 8, dev)
    r1, o1 = serve.run(wl, 8 << 30, closed_loop=True, graphs=True)
    r2, o2 = serve.run(wl, 8 << 30, closed_loop=True, graphs=False)
    assert r1["stats"]["graph_replays"] >= 1 and r2["stats"]["graph_replays"] == 0
    for a, b in zip(o1, o2):
        if a is not None:
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert serve.check(wl, o1)


def test_open_loop_stream_latencies():
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: open-loop Poisson stream")
    reqs = workloads.serving_requests(100, 500.0, 3, build_lo=1 << 10, build_hi=1 << 18,
                                      lookup_lo=1 << 8, lookup_hi=1 << 16)
    wl = serve.Workload(reqs, [10000, 50000], 9, dev)
    res, outs = serve.run(wl, 16 << 30)
    assert res["status_ok"] and serve.check(wl, outs)
    assert 0 < res["lookup_p50_ms"] <= res["lookup_p99_ms"]


def _busy(stream, dev):
    """Queue some tens of milliseconds of device work on `stream` (a bounded chain of
    elementwise kernels), so that whatever follows on it is still pending for a while."""
    import torch
    with torch.cuda.stream(stream):
        x = torch.ones(1 << 25, dtype=torch.float32, device=dev)
        for _ in range(400):
            x = x * 1.0001 + 0.5
    return x


def test_requests_are_ordered_after_the_submitters_stream():
    """Keys and needles written on a side stream behind pending work are submitted at once,
    without any host synchronisation: the server's work waits for that stream, so the map
    equals a standalone build and every needle is answered exactly."""
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: requests ordered after the submitter's stream")
    n = 200000
    side = torch.cuda.Stream()
    keys = torch.empty(n, dtype=torch.int64, device=dev)
    vals = torch.empty(n, dtype=torch.int32, device=dev)
    q = torch.empty(n, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    srv = fks.FksServer(8 << 30)
    _busy(side, dev)
    with torch.cuda.stream(side):
        keys.copy_(workloads.mix_keys_torch(torch.arange(0, n, dtype=torch.int64, device=dev)))
        vals.copy_(torch.arange(n, dtype=torch.int32, device=dev))
        # needles: the keys in reverse order, then keys that are not in the map
        q[: n // 2].copy_(keys[: n // 2].flip(0))
        q[n // 2:].copy_(workloads.mix_keys_torch(torch.arange(n, n + n // 2, dtype=torch.int64, device=dev)))
    _, mid = srv.submit_build(keys, vals, 77, stream=side)
    v = torch.empty(n, dtype=torch.int32, device=dev)
    f = torch.empty(n, dtype=torch.uint8, device=dev)
    srv.submit_lookup(mid, q, v, f, stream=side)
    srv.wait_all()
    torch.cuda.synchronize()
    h1, s1 = export_handle(fks, srv.map_handle(mid))
    alone = fks.fks_build_u64(keys, vals, 77)
    h2, s2, _ = fks.fks_export(alone)
    assert (h1 == h2).all() and (s1 == s2).all()
    want_v = torch.arange(n // 2, dtype=torch.int32, device=dev).flip(0)
    assert bool(f[: n // 2].all()) and not bool(f[n // 2:].any())
    assert torch.equal(v[: n // 2], want_v)
    srv.destroy()


def test_oversized_build_fails_without_evicting():
    """A build whose reservation exceeds the whole budget completes with FKS_ENOMEM at once
    and leaves the resident maps in place."""
    import torch
    fks, serve = _mods()
    dev = torch.device("cuda:0")
    announce("gpu serve: oversized build leaves resident maps alone")
    n = 20000
    per_map = 16 * ((n + 7) // 8) + 16 * 4 * n + 24 * 64 + 4096
    srv = fks.FksServer(3 * per_map)
    ids = []
    for b in range(2):
        k = workloads.mix_keys_torch(torch.arange(b * n, (b + 1) * n, dtype=torch.int64, device=dev))
        v = torch.arange(n, dtype=torch.int32, device=dev)
        ids.append(srv.submit_build(k, v, b + 1)[1])
    srv.wait_all()
    big = 5 * n
    kb = workloads.mix_keys_torch(torch.arange(10 * n, 10 * n + big, dtype=torch.int64, device=dev))
    vb = torch.arange(big, dtype=torch.int32, device=dev)
    rid, _ = srv.submit_build(kb, vb, 9)
    srv.wait_all()
    done, status, _ = srv.poll(rid)
    assert done and status == fks.FKS_ENOMEM
    st = srv.stats()
    assert st["evictions"] == 0 and st["resident_maps"] == 2
    for mid in ids:
        assert srv.map_handle(mid)
    srv.destroy()
