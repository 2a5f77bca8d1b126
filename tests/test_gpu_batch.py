"""GPU parity of the batched build (one persistent launch for many maps) and the
batched lookup, through the C ABI.  Map m of a batch must equal, byte for byte,
the oracle's single-map build with seed = entry m of the batch seed's stream."""
import numpy as np
import pytest

import oracle
from paper_2508_11443_amd import workloads
from tests import fkscheck
from tests.gpu_util import announce, empty, to_dev, to_np

pytestmark = pytest.mark.gpu
MISSING = 0xFFFFFFFF


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def make_batch(sizes, seed):
    sizes = np.asarray(sizes, np.int64)
    off = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    keys = workloads.unique_u64(int(off[-1]), seed, 0.25)
    vals = np.concatenate([np.arange(s, dtype=np.uint32) for s in sizes]) if off[-1] else np.zeros(0, np.uint32)
    return keys, vals, off


def check_map(b, m, keys, vals, off, batch_seed, **kw):
    fks = _fks()
    k = keys[off[m]:off[m + 1]]
    v = vals[off[m]:off[m + 1]]
    ref = oracle.build_u64(k, v, oracle.batch_seed(batch_seed, m), **kw)
    h, s, consts, info = fks.fks_batch_export(b, m)
    rh, rs = ref.export()
    assert info["r"] == ref.r and info["S"] == ref.S, (m, info["r"], ref.r)
    assert (h == rh).all(), f"map {m}: header differs"
    assert (s == rs).all(), f"map {m}: cells differ"
    sizes = fkscheck.decode_header(rh, ref.n)[1][:ref.n] if ref.n else np.zeros(0, np.int64)
    assert info["size_hist"] == np.bincount(sizes, minlength=16).tolist(), f"map {m}: size histogram"


def run_lookup(b, ids, q):
    import torch
    v = empty(q.size, "u32")
    f = empty(q.size, "u8")
    _fks().fks_lookup_batch_u64(b, to_dev(ids.astype(np.uint32)), to_dev(q), v, f, missing=MISSING)
    torch.cuda.synchronize()
    return to_np(v, "u32"), to_np(f, "u8")


def test_small_batch_every_map_bit_exact():
    sizes = [16, 0, 1, 2, 7, 8, 9, 255, 256, 257, 1000, 4096, 5000, 65536, 17, 3000]
    announce(f"gpu batch: {len(sizes)} maps, sizes {sizes}")
    keys, vals, off = make_batch(sizes, 11)
    b = _fks().fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 99)
    st, r, S = b.status()
    assert (st == 0).all()
    for m in range(len(sizes)):
        check_map(b, m, keys, vals, off, 99)
    ids, q, exp_f, exp_v = workloads.batch_queries(keys, off, 20000, 0.75, 5)
    v, f = run_lookup(b, ids, q)
    assert (f == exp_f).all()
    assert (v[exp_f == 1] == exp_v[exp_f == 1]).all()
    assert (v[exp_f == 0] == MISSING).all()


@pytest.mark.parametrize("schedule", [0x10, 0x20, 0x30, 0x11, 0x21, 0x12, 0x110, 0x120, 0x130, 0x111, 0x121, 0x112])
def test_every_schedule_gives_the_same_bytes(schedule):
    """Every schedule builds the same bytes; schedules with bit 0x100 build the maps of
    8192 keys and more with the partition passes (sizes here reach 2^14)."""
    announce(f"gpu batch: schedule {schedule:#x}")
    fks = _fks()
    assert schedule in fks.fks_batch_schedules()
    sizes = workloads.batch_sizes(300, 3, 16, 1 << 14)
    keys, vals, off = make_batch(sizes, 12)
    b0 = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 5, schedule=0x10)
    b1 = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 5, schedule=schedule)
    s0, r0, S0 = b0.status()
    s1, r1, S1 = b1.status()
    assert (s1 == s0).all() and (r1 == r0).all() and (S1 == S0).all()
    for m in range(300):
        a = fks.fks_batch_export(b0, m)
        c = fks.fks_batch_export(b1, m)
        assert (a[0] == c[0]).all() and (a[1] == c[1]).all() and (a[2] == c[2]).all(), m
    big = [m for m in range(300) if off[m + 1] - off[m] >= 8192]
    for m in sorted(set([0, 1, 299] + big[:3])):
        check_map(b1, m, keys, vals, off, 5)


@pytest.mark.parametrize("c,T", [(4, 64), (2, 64), (4, 8)])
def test_wide_maps_with_rejected_attempts(c, T):
    """The partition passes take attempt 0 of every large map; a map they reject is
    rebuilt by the per-workgroup kernel from attempt 0 on.  A space factor of 2 rejects
    about half the attempts on space, a budget of 8 trials about half on exhaustion.
    Every map equals the oracle's build with the same parameters."""
    fks = _fks()
    sizes = [65536, 8192, 8191, 20000, 100, 40000, 9000, 0, 33333, 12000, 15000, 61000]
    announce(f"gpu batch: wide maps, c={c} T={T}")
    keys, vals, off = make_batch(sizes, 14)
    b = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 31, c=c, T=T, R=1024,
                                schedule=0x130)
    st, r, S = b.status()
    assert (st == 0).all()
    for m in range(len(sizes)):
        check_map(b, m, keys, vals, off, 31, c=c, T=T, R=1024)
    if (c, T) != (4, 64):
        assert r.max() > 0   # some large map needed a later attempt
    ids, q, exp_f, exp_v = workloads.batch_queries(keys, off, 50000, 0.75, 9)
    v, f = run_lookup(b, ids, q)
    assert (f == exp_f).all()
    assert (v[exp_f == 1] == exp_v[exp_f == 1]).all()


def test_batch_map_equals_single_map_build():
    import torch
    fks = _fks()
    sizes = [5000, 123, 65536]
    announce("gpu batch: batch map == single-map build")
    keys, vals, off = make_batch(sizes, 13)
    b = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 777)
    for m in range(3):
        k = keys[off[m]:off[m + 1]]
        v = vals[off[m]:off[m + 1]]
        single = fks.fks_build_u64(to_dev(k), to_dev(v), oracle.batch_seed(777, m))
        hs, ss, _ = fks.fks_export(single)
        hb, sb, _, _ = fks.fks_batch_export(b, m)
        assert (hs == hb).all() and (ss == sb).all()
    torch.cuda.synchronize()


def test_failed_map_is_isolated():
    fks = _fks()
    announce("gpu batch: a map with duplicate keys")
    keys, vals, off = make_batch([100, 200, 300], 14)
    keys[off[1] + 5] = keys[off[1] + 9]
    b = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 1)
    st, _, _ = b.status()
    assert st.tolist() == [0, fks.FKS_EDUPKEY, 0]
    # sixteen copies of one key reject every attempt of their map for size; the map
    # reports the repeat, as a single build does, and its neighbours are unaffected
    keys2 = keys.copy()
    keys2[off[1]:off[1] + 16] = keys2[off[1]]
    b2 = fks.fks_build_batch_u64(to_dev(keys2), to_dev(vals), off.astype(np.uint64), 1)
    st2, _, _ = b2.status()
    assert st2.tolist() == [0, fks.FKS_EDUPKEY, 0]
    check_map(b2, 0, keys2, vals, off, 1)
    check_map(b2, 2, keys2, vals, off, 1)
    check_map(b, 0, keys, vals, off, 1)
    check_map(b, 2, keys, vals, off, 1)
    ids = np.array([1, 1, 0, 2, 7], np.uint32)
    q = np.array([keys[off[1] + 5], keys[off[1]], keys[0], keys[off[2]], keys[0]], np.uint64)
    v, f = run_lookup(b, ids, q)
    assert f.tolist() == [0, 0, 1, 1, 0]
    with pytest.raises(fks.FksError) as e:
        fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), np.array([0, 70000], np.uint64), 1)
    assert e.value.code == fks.FKS_EINVAL


def test_forced_retries_in_batch():
    fks = _fks()
    announce("gpu batch: T=1 forces level-one retries")
    keys, vals, off = make_batch([40] * 30, 15)
    b = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 3, T=1, R=1024)
    st, r, _ = b.status()
    assert (st == 0).all() and (r > 0).any()
    for m in range(30):
        check_map(b, m, keys, vals, off, 3, T=1, R=1024)


def test_config4_batch():
    """4096 maps, sizes log-uniform in [16, 2^16], one persistent launch; 2^24 needles at
    75% hits spread over the maps.  Every map byte-exact against the oracle (with its
    bucket-size histogram), every needle against dictionary semantics."""
    fks = _fks()
    M = 4096
    announce(f"gpu batch: config 4, M={M}")
    keys, vals, off = workloads.batch_u64(M, 4)
    b = fks.fks_build_batch_u64(to_dev(keys), to_dev(vals), off.astype(np.uint64), 2024)
    st, r, S = b.status()
    assert (st == 0).all()
    for m in range(M):
        if m % 512 == 0:
            announce(f"gpu batch: config 4, maps {m}..{min(M, m + 512) - 1} against the oracle")
        check_map(b, m, keys, vals, off, 2024)
    ids, q, exp_f, exp_v = workloads.batch_queries(keys, off, 1 << 24, 0.75, 6)
    v, f = run_lookup(b, ids, q)
    assert (f == exp_f).all()
    assert (v[exp_f == 1] == exp_v[exp_f == 1]).all()
