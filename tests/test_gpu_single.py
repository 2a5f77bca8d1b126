"""GPU parity of the single-map path against the CPU oracle, through the C ABI.

Integer work, so the bar is bit-exact: exported header and cell bytes equal the
oracle's, lookup values and found flags equal the oracle's (and dictionary
semantics).  Sizes span several search blocks (256 buckets) and scan tiles
(2048 groups) with ragged tails; the full 2^26-key bench configuration is built
and compared byte for byte."""
import numpy as np
import pytest

import oracle
from paper_2508_11443_amd import workloads
from tests import collide, fkscheck
from tests.gpu_util import announce, empty, to_dev, to_np

pytestmark = pytest.mark.gpu

MISSING = 0xDEADBEEF


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def gpu_build(keys, vals, seed, **kw):
    return _fks().fks_build_u64(to_dev(keys), to_dev(vals), seed, **kw)


def gpu_lookup(m, q):
    import torch
    fks = _fks()
    v = empty(q.size, "u32")
    f = empty(q.size, "u8")
    fks.fks_lookup_u64(m, to_dev(q), v, f, missing=MISSING)
    torch.cuda.synchronize()
    return to_np(v, "u32"), to_np(f, "u8")


def assert_same_table(m, ref):
    h, s, consts = _fks().fks_export(m)
    rh, rs = ref.export()
    inf = m.info()
    assert inf["r"] == ref.r and inf["S"] == ref.S and inf["n"] == ref.n
    assert h.size == rh.size and (h == rh).all(), "header bytes differ"
    assert s.size == rs.size and (s == rs).all(), "cell bytes differ"
    # the bucket-size histogram of fks_info counts the oracle's sizes of the n buckets
    sizes = fkscheck.decode_header(rh, ref.n)[1][:ref.n] if ref.n else np.zeros(0, np.int64)
    assert inf["size_hist"] == np.bincount(sizes, minlength=16).tolist()


SIZES = [1, 2, 3, 7, 8, 9, 63, 255, 256, 257, 1000, 2047, 2048 * 8 + 5, 65536, 100003, (1 << 20) + 77]


@pytest.mark.parametrize("n", SIZES)
def test_build_and_lookup_bit_exact(n):
    seed = 0x5EED + n
    announce(f"gpu single u64: n={n} seed={seed}")
    keys = workloads.unique_u64(n, n, dense_fraction=0.5)
    vals = (np.arange(n, dtype=np.uint64) * 0x9E3779B1 % (1 << 32)).astype(np.uint32)
    m = gpu_build(keys, vals, seed)
    ref = oracle.build_u64(keys, vals, seed)
    assert_same_table(m, ref)
    q, expect = workloads.u64_queries(keys, max(2 * n, 1000), 0.5, n + 1)
    v, f = gpu_lookup(m, q)
    rv, rf = ref.lookup(q, missing=MISSING)
    assert (f == rf).all() and (rf == expect).all()
    assert (v == rv).all()


def test_empty_map():
    import torch
    announce("gpu single u64: empty map")
    m = gpu_build(np.zeros(0, np.uint64), np.zeros(0, np.uint32), 3)
    assert m.info()["n"] == 0 and m.info()["S"] == 0
    q = np.array([0, 1, 2**64 - 1], np.uint64)
    v, f = gpu_lookup(m, q)
    assert f.tolist() == [0, 0, 0] and v.tolist() == [MISSING] * 3
    # m = 0 lookups are a no-op
    _fks().fks_lookup_u64(m, to_dev(np.zeros(0, np.uint64)), empty(0, "u32"), empty(0, "u8"))
    torch.cuda.synchronize()


def test_contains_and_optional_outputs():
    import torch
    announce("gpu single u64: contains / value-only lookups")
    n = 50000
    keys = workloads.unique_u64(n, 5, 0.5)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build(keys, vals, 9)
    q, expect = workloads.u64_queries(keys, 3 * n, 0.5, 6)
    f = empty(q.size, "u8")
    _fks().fks_contains_u64(m, to_dev(q), f)
    v = empty(q.size, "u32")
    _fks().fks_lookup_u64(m, to_dev(q), v, None, missing=7)
    torch.cuda.synchronize()
    ref = oracle.build_u64(keys, vals, 9)
    rv, rf = ref.lookup(q, missing=7)
    assert (to_np(f, "u8") == rf).all()
    assert (to_np(v, "u32") == rv).all()


def test_deterministic_and_order_independent():
    announce("gpu single u64: determinism")
    n = 300001
    keys = workloads.unique_u64(n, 77, 0.5)
    vals = np.arange(n, dtype=np.uint32)
    a = _fks().fks_export(gpu_build(keys, vals, 1))
    b = _fks().fks_export(gpu_build(keys, vals, 1))
    perm = np.random.default_rng(3).permutation(n)
    c = _fks().fks_export(gpu_build(keys[perm], vals[perm], 1))
    for x, y in ((a, b), (a, c)):
        assert (x[0] == y[0]).all() and (x[1] == y[1]).all()


def test_forced_retries_match_oracle():
    announce("gpu single u64: forced level-one retries (T=1, c=2)")
    keys = workloads.unique_u64(3000, 8)
    vals = np.arange(3000, dtype=np.uint32)
    retried = 0
    for seed in range(12):
        m = gpu_build(keys[:40], vals[:40], seed, T=1, R=1024)
        ref = oracle.build_u64(keys[:40], vals[:40], seed, T=1, R=1024)
        assert_same_table(m, ref)
        retried += ref.r > 0
    assert retried > 0
    for seed in range(6):
        m = gpu_build(keys[:500], vals[:500], seed, c=2, R=64)
        ref = oracle.build_u64(keys[:500], vals[:500], seed, c=2, R=64)
        assert_same_table(m, ref)


@pytest.mark.parametrize("s", [8, 12])
def test_late_trial_bucket_bit_exact(s):
    """A bucket that no trial below 16 separates (crafted keys, tests/late_trials.py): its
    search and placement read triples beyond those the final pass stages in LDS (the search of
    a bucket of at most 8 keys, and of a larger one)."""
    from tests import late_trials
    sigma, n = 0x1A7E, 1024
    announce(f"gpu single u64: late trial, bucket of {s} keys, n={n}")
    keys = late_trials.keys_with_late_trial(sigma, n, s)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.build_u64(keys, vals, sigma)
    assert fkscheck.decode_header(ref.export()[0], n)[2][0] >= 16
    m = gpu_build(keys, vals, sigma)
    assert_same_table(m, ref)
    assert m.info()["max_t"] >= 16
    v, f = gpu_lookup(m, keys)
    assert f.all() and (v == vals).all()


def test_errors():
    fks = _fks()
    announce("gpu single u64: error paths")
    keys = workloads.unique_u64(1000, 4)
    keys[10] = keys[500]
    with pytest.raises(fks.FksError) as e:
        gpu_build(keys, np.zeros(1000, np.uint32), 1)
    assert e.value.code == fks.FKS_EDUPKEY
    # every attempt rejected (a bucket above 15 keys, or too many cells): repeated keys
    # are reported as such, on both schedules, as the oracle reports them
    for keys_r, kw in ((np.full(16, 9, np.uint64), {}), (np.full(16, 9, np.uint64), {"schedule": 1}),
                       (np.repeat(workloads.unique_u64(300, 7), 10), {})):
        with pytest.raises(oracle.OracleError) as eo:
            oracle.build_u64(keys_r, np.zeros(keys_r.size, np.uint32), 1)
        with pytest.raises(fks.FksError) as e:
            gpu_build(keys_r, np.zeros(keys_r.size, np.uint32), 1, **kw)
        assert e.value.code == fks.FKS_EDUPKEY == eo.value.code
    with pytest.raises(fks.FksError) as e:
        fks.fks_build_u64_v64(to_dev(np.full(20, 3, np.uint64)), to_dev(np.zeros(20, np.uint64)), 1)
    assert e.value.code == fks.FKS_EDUPKEY
    with pytest.raises(fks.FksError) as e:
        gpu_build(workloads.unique_u64(2000, 1), np.zeros(2000, np.uint32), 1, c=1)
    assert e.value.code == fks.FKS_EBUILD
    with pytest.raises(fks.FksError) as e:
        gpu_build(np.arange(5, dtype=np.uint64), np.zeros(5, np.uint32), 1, T=300)
    assert e.value.code == fks.FKS_EINVAL
    # a map of integer keys refuses string needles
    m = gpu_build(np.arange(5, dtype=np.uint64), np.zeros(5, np.uint32), 1)
    off = to_dev(np.array([0, 1], np.int64))
    with pytest.raises(fks.FksError) as e:
        fks.fks_lookup_bytes(m, off, to_dev(np.array([65], np.uint8)), empty(1, "u32"), empty(1, "u8"))
    assert e.value.code == fks.FKS_EINVAL


def test_bench_size_bit_exact():
    """The 2^26-key configuration (half uniform, half one dense run), in the launch
    configuration the benchmark times, against the oracle byte for byte; lookups of
    2^26 needles at 50% hits against dictionary semantics."""
    import torch
    n = 1 << 26
    seed = 0xF00D
    announce(f"gpu single u64: bench size n={n}")
    keys = workloads.unique_u64(n, 2026, dense_fraction=0.5)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build(keys, vals, seed)
    ref = oracle.build_u64(keys, vals, seed)
    assert_same_table(m, ref)
    q, expect, src = workloads.u64_queries(keys, n, 0.5, 2027, return_index=True)
    v, f = gpu_lookup(m, q)
    assert (f == expect).all()
    hit = expect == 1
    # the value of a hit is the index of its key
    assert (v[hit] == src[hit].astype(np.uint32)).all()
    assert (v[~hit] == MISSING).all()
    del m
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [100000, 300000])
def test_crowded_partition_takes_the_counted_passes(n):
    """With 1024 < n <= 2^26 keys the build reserves each partition's records in a region of
    fixed capacity (about 1.5x the 1024 keys a partition holds on average), in one pass
    (n = 100000) or two (n = 300000).  Here over 2000 keys hash (under attempt 0's level-one
    constants) into the first partition's 1024 buckets: its region overflows and the attempt
    is redone with counted passes.  The table must still equal the oracle's byte for byte."""
    from oracle import rounds, spec
    seed = 0xC20D
    announce(f"gpu single u64: crowded first partition, n={n} seed={seed}")
    a0, a1, b, _ = spec.level1_consts(seed, 0)
    rng = np.random.default_rng(99)
    crowd = np.zeros(0, np.uint64)
    while crowd.size < 2100:
        cand = rng.integers(0, 1 << 64, size=1 << 22, dtype=np.uint64)
        crowd = np.unique(np.concatenate([crowd, cand[rounds.hash_vec(a0, a1, b, cand) % n < 1024]]))
    crowd = crowd[:2100]
    rest = workloads.unique_u64(n, 7, dense_fraction=0.0)
    rest = rest[~np.isin(rest, crowd)][:n - crowd.size]
    keys = np.concatenate([crowd, rest])
    assert np.unique(keys).size == n
    assert (rounds.hash_vec(a0, a1, b, keys) % n < 1024).sum() > 2000
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.build_u64(keys, vals, seed)
    assert ref.r == 0
    m = gpu_build(keys, vals, seed)
    assert_same_table(m, ref)
    q, expect, src = workloads.u64_queries(keys, 1 << 16, 0.5, 5, return_index=True)
    v, f = gpu_lookup(m, q)
    assert (f == expect).all() and (v[expect == 1] == src[expect == 1].astype(np.uint32)).all()


@pytest.mark.parametrize("n", [(1 << 26) + 1, (1 << 27) + 12345])
def test_three_radix_passes_bit_exact(n):
    """More than 2^16 partitions of 1024 buckets: the partition index is grouped in three
    radix passes of at most 8 bits each (2^26 + 1 keys is the smallest such build).  The
    table equals the oracle's byte for byte; sampled lookups equal the oracle's."""
    seed = 0x3A55 + n
    announce(f"gpu single u64: three radix passes, n={n}")
    keys = workloads.unique_u64(n, n + 5, dense_fraction=0.25)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build(keys, vals, seed)
    ref = oracle.build_u64(keys, vals, seed)
    assert_same_table(m, ref)
    rng = np.random.default_rng(n)
    q = np.concatenate([keys[rng.integers(0, n, size=50000)],
                        rng.integers(0, 2**64, size=50000, dtype=np.uint64, endpoint=False)])
    v, f = gpu_lookup(m, q)
    rv, rf = ref.lookup(q, missing=MISSING)
    assert (f == rf).all() and (v == rv).all()
    del m, ref


# ---- attempts with unusual bucket sizes ------------------------------------------------

def skewed_keys(n, seed, per_bucket, rng_seed, big=0):
    """n distinct keys whose level-one buckets under attempt 0 of `seed` (the oracle's
    constants) are mostly every per_bucket-th bucket, per_bucket keys each, so that S is
    near per_bucket * n; with big > 0, bucket 1 receives `big` keys as well."""
    a0, a1, b, _ = oracle.level1_consts(seed, 0)
    rng = np.random.default_rng(rng_seed)
    pool = np.unique(rng.integers(0, 2**64, size=(14 + 3 * big) * n, dtype=np.uint64))
    pool = rng.permutation(pool)
    with np.errstate(over="ignore"):
        h = (np.uint64(a0) * (pool & np.uint64(0xFFFFFFFF)) + np.uint64(a1) * (pool >> np.uint64(32)) +
             np.uint64(b)) >> np.uint64(32)
    j = (h % np.uint64(n)).astype(np.int64)
    picked = []
    if big:
        picked.append(pool[j == 1][:big])
        assert picked[0].size == big
    in_b = (j % per_bucket == 0) & (j != 1)
    kb, jb = pool[in_b], j[in_b]
    order = np.argsort(jb, kind="stable")
    kb, jb = kb[order], jb[order]
    first = np.searchsorted(jb, jb, side="left")
    rank = np.arange(jb.size) - first
    picked.append(kb[rank < per_bucket])
    keys = np.concatenate(picked)[: n]
    if keys.size < n:   # top up with keys of other buckets
        rest = pool[~in_b & (j != 1)]
        keys = np.concatenate([keys, rest[: n - keys.size]])
    assert keys.size == n and np.unique(keys).size == n
    return rng.permutation(keys)


@pytest.mark.parametrize("n", [6000, 100003])
def test_more_cells_than_the_first_allocation(n):
    """Buckets of three keys in a third of the buckets: S is near 3n, above the cells the
    build allocates before its final pass (about 2n), so the pass runs again into an
    exact allocation.  Attempt 0 is accepted (S <= 4n); table bytes equal the oracle's."""
    seed = 0xB16 + n
    announce(f"gpu single u64: S above the first allocation, n={n}")
    keys = skewed_keys(n, seed, 3, n)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.build_u64(keys, vals, seed)
    assert ref.r == 0 and ref.S > 2.5 * n
    m = gpu_build(keys, vals, seed)
    assert_same_table(m, ref)
    q, _ = workloads.u64_queries(keys, 3000, 0.5, 9)
    v, f = gpu_lookup(m, q)
    rv, rf = ref.lookup(q, missing=MISSING)
    assert (f == rf).all() and (v == rv).all()


@pytest.mark.parametrize("case", ["oversize", "space"])
def test_rejected_first_attempt(case):
    """Attempt 0 rejected inside the final pass: a bucket of 16 keys (oversize), or S near
    3n with c = 2 (space).  The next attempt is accepted; bytes equal the oracle's."""
    n = 50000
    seed = 0x0DD + len(case)
    announce(f"gpu single u64: first attempt rejected ({case})")
    if case == "oversize":
        keys, kw = skewed_keys(n, seed, 1, 77, big=16), {}
    else:
        keys, kw = skewed_keys(n, seed, 3, 78), {"c": 2}
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.build_u64(keys, vals, seed, **kw)
    assert ref.r >= 1
    m = gpu_build(keys, vals, seed, **kw)
    assert_same_table(m, ref)


# ---- string keys ---------------------------------------------------------------------

def gpu_build_bytes(off, data, vals, seed, **kw):
    return _fks().fks_build_bytes(to_dev(off), to_dev(data), to_dev(vals), seed, **kw)


@pytest.mark.parametrize("n", [1, 2, 50, 257, 3000, 100000])
def test_string_map_bit_exact(n):
    import torch
    seed = 31 + n
    announce(f"gpu single bytes: n={n} seed={seed}")
    off, data = workloads.random_strings(n, 17 + n)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build_bytes(off, data, vals, seed)
    ref = oracle.build_bytes(off, data, vals, seed)
    assert_same_table(m, ref)
    qo, qd, qf, qi = workloads.string_queries(off, data, 2 * n + 10, 0.5, 5)
    v = empty(qo.size - 1, "u32")
    f = empty(qo.size - 1, "u8")
    _fks().fks_lookup_bytes(m, to_dev(qo), to_dev(qd), v, f, missing=MISSING)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_bytes(qo, qd, missing=MISSING)
    assert (to_np(f, "u8") == rf).all() and (rf == qf).all()
    assert (to_np(v, "u32") == rv).all()


def test_fingerprint_collision_takes_the_next_attempt():
    """Two distinct 16-byte strings whose fingerprints are equal under attempt 0's base share
    a bucket no level-two trial can split: the GPU build must reject attempt 0 (the strings
    differ, so this is no repeated key), take attempt 1 with its new base, and export the
    oracle's bytes; every string, the two included, is found with its value."""
    import torch
    sigma = 0xC0111DE
    announce(f"gpu single bytes: fingerprint collision under attempt 0, seed={sigma}")
    for n_other in (3000, 1):
        off, data, a, b = collide.strings_with_collision(sigma, n_other, 77)
        n = off.size - 1
        vals = np.arange(n, dtype=np.uint32)
        ref = oracle.build_bytes(off, data, vals, sigma)
        assert ref.r >= 1 and ref.info["rejected_exhausted"] >= 1
        m = gpu_build_bytes(off, data, vals, sigma)
        assert_same_table(m, ref)
        v = empty(n, "u32")
        f = empty(n, "u8")
        _fks().fks_lookup_bytes(m, to_dev(off), to_dev(data), v, f, missing=MISSING)
        torch.cuda.synchronize()
        assert to_np(f, "u8").all() and (to_np(v, "u32") == vals).all()


def test_string_bench_size_bit_exact():
    """The string configuration at full size: 2^22 unique lowercase strings of 4..64 bytes
    (as the benchmark builds them), table bytes against the oracle, 2^22 needles at 50 %
    hits against the oracle and dictionary semantics."""
    import torch
    n = 1 << 22
    announce(f"gpu single bytes: bench size n={n}")
    off, data = workloads.random_strings(n, 303)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build_bytes(off, data, vals, 7)
    ref = oracle.build_bytes(off, data, vals, 7)
    assert_same_table(m, ref)
    qo, qd, qf, _ = workloads.string_queries(off, data, n, 0.5, 304)
    v = empty(n, "u32")
    f = empty(n, "u8")
    _fks().fks_lookup_bytes(m, to_dev(qo), to_dev(qd), v, f, missing=MISSING)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_bytes(qo, qd, missing=MISSING)
    assert (to_np(f, "u8") == rf).all() and (rf == qf).all()
    assert (to_np(v, "u32") == rv).all()


def test_string_lengths_across_chunks():
    """Strings of 0..300 arbitrary bytes (the kernels read them 64 bytes at a time as
    aligned words, so lengths around multiples of 64 and every byte alignment matter):
    table bytes against the oracle; needles are every key, and every key with its first or
    last byte changed, one byte shorter or one byte longer."""
    import torch
    rng = np.random.default_rng(12)
    lens = rng.integers(0, 301, size=3000)
    strings = [bytes(rng.integers(0, 256, size=int(L), dtype=np.uint8)) for L in lens]
    strings += [b"x" * L for L in (4, 63, 64, 65, 127, 128, 129, 191, 192, 193)]
    strings = list(dict.fromkeys(strings))
    announce(f"gpu single bytes: lengths 0..300, {len(strings)} strings")
    off, data = workloads.to_csr(strings)
    vals = np.arange(len(strings), dtype=np.uint32)
    m = gpu_build_bytes(off, data, vals, 77)
    ref = oracle.build_bytes(off, data, vals, 77)
    assert_same_table(m, ref)
    needles = list(strings)
    for x in strings[:800]:
        if x:
            needles.append(bytes([x[0] ^ 1]) + x[1:])
            needles.append(x[:-1] + bytes([x[-1] ^ 0x80]))
            needles.append(x[:-1])
        needles.append(x + b"q")
    qo, qd = workloads.to_csr(needles)
    v = empty(len(needles), "u32")
    f = empty(len(needles), "u8")
    _fks().fks_lookup_bytes(m, to_dev(qo), to_dev(qd), v, f, missing=MISSING)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_bytes(qo, qd, missing=MISSING)
    assert (to_np(f, "u8") == rf).all() and (to_np(v, "u32") == rv).all()
    d = {x: i for i, x in enumerate(strings)}
    assert to_np(f, "u8").tolist() == [1 if x in d else 0 for x in needles]


def test_string_map_edge_cases():
    import torch
    fks = _fks()
    announce("gpu single bytes: empty strings, duplicates, bad offsets")
    strings = [b"", b"a", b"ab", b"abc", b"abcd", b"abcde", b"\0", b"a\0"]
    off, data = workloads.to_csr(strings)
    vals = np.arange(len(strings), dtype=np.uint32)
    m = gpu_build_bytes(off, data, vals, 4)
    ref = oracle.build_bytes(off, data, vals, 4)
    assert_same_table(m, ref)
    qo, qd = workloads.to_csr(strings + [b"abcdef", b"\0\0", b"b"])
    v = empty(qo.size - 1, "u32")
    f = empty(qo.size - 1, "u8")
    fks.fks_lookup_bytes(m, to_dev(qo), to_dev(qd), v, f, missing=MISSING)
    torch.cuda.synchronize()
    assert to_np(f, "u8").tolist() == [1] * 8 + [0] * 3
    assert to_np(v, "u32").tolist()[:8] == list(range(8))
    # needle offsets that are not a range of the needle buffer are answered absent and
    # nothing is read through them: a negative start, an end before the start, an end past
    # the buffer; the well-formed needles around them are answered as usual
    buf = np.frombuffer(b"abcabcd", np.uint8)
    qo = np.array([0, 3, -5, 7, 2, 10**12, 3, 7], np.int64)
    v = empty(qo.size - 1, "u32")
    f = empty(qo.size - 1, "u8")
    fks.fks_lookup_bytes(m, to_dev(qo), to_dev(buf), v, f, missing=MISSING)
    torch.cuda.synchronize()
    assert to_np(f, "u8").tolist() == [1, 0, 0, 0, 0, 0, 1]
    assert to_np(v, "u32").tolist() == [3, MISSING, MISSING, MISSING, MISSING, MISSING, 4]
    dup_off, dup_data = workloads.to_csr([b"alpha", b"beta", b"gamma", b"beta"])
    with pytest.raises(fks.FksError) as e:
        gpu_build_bytes(dup_off, dup_data, np.zeros(4, np.uint32), 1)
    assert e.value.code == fks.FKS_EDUPKEY
    # sixteen copies of one string: every attempt is rejected for size, then the equal-key
    # check reports them (strings equal on a prefix are not repeats)
    rep_off, rep_data = workloads.to_csr([b"same"] * 16 + [b"sam", b"samee", b"other"])
    with pytest.raises(fks.FksError) as e:
        gpu_build_bytes(rep_off, rep_data, np.zeros(19, np.uint32), 1)
    assert e.value.code == fks.FKS_EDUPKEY
    pre_off, pre_data = workloads.to_csr([b"ab" * k for k in range(1, 17)])
    pm = gpu_build_bytes(pre_off, pre_data, np.arange(16, dtype=np.uint32), 1)
    assert_same_table(pm, oracle.build_bytes(pre_off, pre_data, np.arange(16, dtype=np.uint32), 1))
    bad = np.array([0, 5, 3, 9], np.int64)
    with pytest.raises(fks.FksError) as e:
        gpu_build_bytes(bad, np.zeros(9, np.uint8), np.zeros(3, np.uint32), 1)
    assert e.value.code == fks.FKS_EINVAL
    e0 = gpu_build_bytes(np.zeros(1, np.int64), np.zeros(0, np.uint8), np.zeros(0, np.uint32), 1)
    assert e0.info()["n"] == 0


# ---- from_array: repeated keys ---------------------------------------------------------

@pytest.mark.parametrize("u,distinct", [(1, 1), (10, 3), (5000, 1000), (300000, 100000), (1 << 20, 1 << 16)])
def test_from_array_bit_exact(u, distinct):
    """Repeated keys keep the value of their first occurrence; the table equals the oracle's
    from_array (dedup, then from_array_nodup)."""
    rng = np.random.default_rng(u)
    pool = workloads.unique_u64(distinct, u + 3)
    if distinct > 2:
        pool[1] = np.uint64(2**64 - 1)       # the all-ones key is handled beside the table
    keys = pool[rng.integers(0, distinct, size=u)]
    vals = rng.integers(0, 2**32, size=u, dtype=np.uint64).astype(np.uint32)
    seed = 99 + u
    announce(f"gpu from_array: u={u} distinct~{distinct}")
    m = _fks().fks_build_u64_from_array(to_dev(keys), to_dev(vals), seed)
    ref = oracle.build_u64_dedup(keys, vals, seed)
    assert_same_table(m, ref)
    q, _ = workloads.u64_queries(np.unique(keys), 2000, 0.5, 5)
    v, f = gpu_lookup(m, q)
    rv, rf = ref.lookup(q, missing=MISSING)
    assert (f == rf).all() and (v == rv).all()
    # first occurrence wins
    first = {}
    for k, val in zip(keys.tolist(), vals.tolist()):
        first.setdefault(k, val)
    hit = f == 1
    assert all(first[int(k)] == int(x) for k, x in zip(q[hit], v[hit]))


# ---- the paper's flattened rounds as the level-two schedule ------------------------------

@pytest.mark.parametrize("n", [1, 2, 9, 1000, 65536, 100003, (1 << 20) + 77])
def test_rounds_schedule_bit_exact(n):
    """schedule=1 searches level two with the sortless rounds of Section 2.5 on the GPU; the
    table must equal the oracle's (and so the per-bucket schedule's) byte for byte."""
    seed = 0xACE + n
    announce(f"gpu rounds schedule: n={n} seed={seed}")
    keys = workloads.unique_u64(n, 3 * n + 1, dense_fraction=0.5)
    vals = np.arange(n, dtype=np.uint32)
    m = gpu_build(keys, vals, seed, schedule=1)
    ref = oracle.build_u64(keys, vals, seed)
    assert_same_table(m, ref)


def test_rounds_schedule_retries_and_duplicates():
    fks = _fks()
    announce("gpu rounds schedule: T=1 retries, duplicate keys")
    keys = workloads.unique_u64(3000, 8)
    vals = np.arange(3000, dtype=np.uint32)
    for seed in range(8):
        m = gpu_build(keys[:40], vals[:40], seed, T=1, R=1024, schedule=1)
        ref = oracle.build_u64(keys[:40], vals[:40], seed, T=1, R=1024)
        assert_same_table(m, ref)
    dup = keys[:1000].copy()
    dup[10] = dup[500]
    with pytest.raises(fks.FksError) as e:
        gpu_build(dup, vals[:1000], 1, schedule=1)
    assert e.value.code == fks.FKS_EDUPKEY


# ---- 64-bit values -------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 9, 1000, 5000, 300007, (1 << 20) + 77])
def test_u64_values_bit_exact(n):
    """Maps with 64-bit values: the scatter passes carry the high halves as aux
    words (0, 1 and 2 passes across these sizes); table bytes and lookups equal
    the oracle's."""
    import torch
    fks = _fks()
    seed = 0x64 + n
    announce(f"gpu single u64v64: n={n} seed={seed}")
    keys = workloads.unique_u64(n, n + 5, dense_fraction=0.5)
    vals = np.random.default_rng(n).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    m = fks.fks_build_u64_v64(to_dev(keys), to_dev(vals), seed)
    ref = oracle.build_u64_v64(keys, vals, seed)
    assert m.info()["kind"] == 2
    assert_same_table(m, ref)
    q, expect = workloads.u64_queries(keys, max(2 * n, 1000), 0.5, n + 2)
    v = empty(q.size, "u64")
    f = empty(q.size, "u8")
    fks.fks_lookup_u64_v64(m, to_dev(q), v, f, missing=2**64 - 7)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_v64(q, missing=2**64 - 7)
    assert (to_np(f, "u8") == rf).all() and (rf == expect).all()
    assert (to_np(v, "u64") == rv).all()
    # membership works on this kind; 32-bit lookups are refused
    f2 = empty(q.size, "u8")
    fks.fks_contains_u64(m, to_dev(q), f2)
    torch.cuda.synchronize()
    assert (to_np(f2, "u8") == rf).all()
    with pytest.raises(fks.FksError) as e:
        fks.fks_lookup_u64(m, to_dev(q), empty(q.size, "u32"), f)
    assert e.value.code == fks.FKS_EINVAL


def test_u64_values_empty_map():
    import torch
    fks = _fks()
    announce("gpu single u64v64: empty map")
    m = fks.fks_build_u64_v64(to_dev(np.zeros(0, np.uint64)), to_dev(np.zeros(0, np.uint64)), 3)
    q = np.array([0, 1, 2**64 - 1], np.uint64)
    v = empty(3, "u64")
    f = empty(3, "u8")
    fks.fks_lookup_u64_v64(m, to_dev(q), v, f, missing=42)
    torch.cuda.synchronize()
    assert (to_np(v, "u64") == 42).all() and not to_np(f, "u8").any()
