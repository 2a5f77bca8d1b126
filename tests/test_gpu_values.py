"""GPU parity of map and reduce over a map's values, through the C ABI.

fks_map_values must give byte for byte the table the oracle builds for the pairs (k, f(v)),
on maps with 32-bit values, 64-bit values and string keys, at sizes spanning many groups with
a ragged tail.  fks_reduce_values must equal the oracle's fold over the input values (each key
once: the fill copies in the table are not values), including the empty map's identities."""
import numpy as np
import pytest

import oracle
from oracle import values as ov
from paper_2508_11443_amd import workloads
from tests.gpu_util import announce, empty, to_dev, to_np

pytestmark = pytest.mark.gpu

OPS = [(ov.VOP_ADD, 0x12345678ABCDEF01, 0), (ov.VOP_MUL, 0x9E3779B97F4A7C15, 0),
       (ov.VOP_XOR, 0xFFFF0000FFFF0000, 0), (ov.VOP_AFFINE, 0x2545F4914F6CDD1D, 0x8BADF00D)]


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def _same_table(m, ref):
    h, s, _ = _fks().fks_export(m)
    rh, rs = ref.export()
    inf = m.info()
    assert inf["r"] == ref.r and inf["S"] == ref.S and inf["n"] == ref.n
    assert h.size == rh.size and (h == rh).all(), "header bytes differ"
    assert s.size == rs.size and (s == rs).all(), "cell bytes differ"


def _u64_case(n, seed):
    keys = workloads.unique_u64(n, seed, dense_fraction=0.5)
    vals = np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return keys, vals


@pytest.mark.parametrize("n", [1, 9, 1000, 100003])
@pytest.mark.parametrize("op,a,b", OPS)
def test_map_values_u32_bit_exact(n, op, a, b):
    fks = _fks()
    seed = 0x7A1 + n
    announce(f"gpu map_values u32: n={n} op={op}")
    keys, vals = _u64_case(n, n + 3)
    m = fks.fks_build_u64(to_dev(keys), to_dev(vals), seed)
    m2 = fks.fks_map_values(m, op, a, b)
    ref = oracle.build_u64(keys, ov.map_values(vals, op, a, b, width=32), seed)
    _same_table(m2, ref)
    # the source map is unchanged
    _same_table(m, oracle.build_u64(keys, vals, seed))


@pytest.mark.parametrize("n", [1, 5000, 300007])
@pytest.mark.parametrize("op,a,b", OPS)
def test_map_values_u64_bit_exact(n, op, a, b):
    import torch
    fks = _fks()
    seed = 0x7A2 + n
    announce(f"gpu map_values u64v64: n={n} op={op}")
    keys = workloads.unique_u64(n, n + 4, dense_fraction=0.5)
    vals = np.random.default_rng(n).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    m = fks.fks_build_u64_v64(to_dev(keys), to_dev(vals), seed)
    m2 = fks.fks_map_values(m, op, a, b)
    mapped = ov.map_values(vals, op, a, b, width=64)
    ref = oracle.build_u64_v64(keys, mapped, seed)
    _same_table(m2, ref)
    q, expect = workloads.u64_queries(keys, max(2 * n, 1000), 0.5, n + 9)
    v = empty(q.size, "u64")
    f = empty(q.size, "u8")
    fks.fks_lookup_u64_v64(m2, to_dev(q), v, f, missing=3)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_v64(q, missing=3)
    assert (to_np(f, "u8") == rf).all() and (rf == expect).all()
    assert (to_np(v, "u64") == rv).all()


@pytest.mark.parametrize("n", [3, 20000])
def test_map_values_strings_bit_exact(n):
    import torch
    fks = _fks()
    seed = 0x7A3 + n
    announce(f"gpu map_values bytes: n={n}")
    off, data = workloads.random_strings(n, 23 + n)
    vals = np.arange(n, dtype=np.uint32)
    m = fks.fks_build_bytes(to_dev(off), to_dev(data), to_dev(vals), seed)
    table = np.random.default_rng(n).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    m2 = fks.fks_map_values(m, fks.FKS_VOP_GATHER, table=to_dev(table))
    ref = oracle.build_bytes(off, data, ov.map_values(vals, ov.VOP_GATHER, table=table), seed)
    _same_table(m2, ref)
    # the new map holds its own context: it still answers after the source map is gone
    m.destroy()
    qo, qd, qf, _ = workloads.string_queries(off, data, 2 * n + 10, 0.5, 8)
    v = empty(qo.size - 1, "u32")
    f = empty(qo.size - 1, "u8")
    fks.fks_lookup_bytes(m2, to_dev(qo), to_dev(qd), v, f, missing=7)
    torch.cuda.synchronize()
    rv, rf = ref.lookup_bytes(qo, qd, missing=7)
    assert (to_np(f, "u8") == rf).all() and (rf == qf).all()
    assert (to_np(v, "u32") == rv).all()


def test_map_values_chain_and_empty_map():
    fks = _fks()
    announce("gpu map_values: add then its inverse; empty map")
    keys, vals = _u64_case(4099, 11)
    m = fks.fks_build_u64(to_dev(keys), to_dev(vals), 5)
    a = 0x0F1E2D3C
    back = fks.fks_map_values(fks.fks_map_values(m, fks.FKS_VOP_ADD, a), fks.FKS_VOP_ADD, (1 << 32) - a)
    _same_table(back, oracle.build_u64(keys, vals, 5))
    e = fks.fks_build_u64(to_dev(np.zeros(0, np.uint64)), to_dev(np.zeros(0, np.uint32)), 5)
    e2 = fks.fks_map_values(e, fks.FKS_VOP_MUL, 3)
    assert e2.info()["n"] == 0 and e2.info()["S"] == 0


def test_map_values_gather_outside_the_table_is_refused():
    fks = _fks()
    announce("gpu map_values: gather index outside the table")
    keys = workloads.unique_u64(500, 12)
    vals = np.arange(500, dtype=np.uint32)
    m = fks.fks_build_u64(to_dev(keys), to_dev(vals), 6)
    with pytest.raises(fks.FksError) as err:
        fks.fks_map_values(m, fks.FKS_VOP_GATHER, table=to_dev(np.zeros(499, np.uint32)))
    assert err.value.code == fks.FKS_EINVAL
    with pytest.raises(fks.FksError) as err:
        fks.fks_map_values(m, 9)
    assert err.value.code == fks.FKS_EINVAL
    # a table that covers every value succeeds, and the source map still works
    m2 = fks.fks_map_values(m, fks.FKS_VOP_GATHER, table=to_dev(np.arange(500, dtype=np.uint32) * 2))
    _same_table(m2, oracle.build_u64(keys, vals * 2, 6))
    _same_table(m, oracle.build_u64(keys, vals, 6))


REDS = [ov.VRED_SUM, ov.VRED_MIN, ov.VRED_MAX, ov.VRED_XOR]


@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 1000, 100003, (1 << 20) + 77])
def test_reduce_values_u32(n):
    fks = _fks()
    announce(f"gpu reduce_values u32: n={n}")
    keys, vals = _u64_case(n, n + 21)
    m = fks.fks_build_u64(to_dev(keys), to_dev(vals), 0x9D + n)
    for op in REDS:
        assert fks.fks_reduce_values(m, op) == ov.reduce_values(vals, op, 32), op


@pytest.mark.parametrize("n", [0, 3, 5000, 300007])
def test_reduce_values_u64(n):
    fks = _fks()
    announce(f"gpu reduce_values u64v64: n={n}")
    keys = workloads.unique_u64(n, n + 22)
    vals = np.random.default_rng(n + 1).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    m = fks.fks_build_u64_v64(to_dev(keys), to_dev(vals), 0x9E + n)
    for op in REDS:
        assert fks.fks_reduce_values(m, op) == ov.reduce_values(vals, op, 64), op


def test_reduce_values_strings_and_device_output():
    import torch
    fks = _fks()
    announce("gpu reduce_values bytes, device output on a side stream")
    off, data = workloads.random_strings(30000, 41)
    vals = np.random.default_rng(41).integers(0, 1 << 32, size=30000, dtype=np.uint64).astype(np.uint32)
    m = fks.fks_build_bytes(to_dev(off), to_dev(data), to_dev(vals), 77)
    side = torch.cuda.Stream()
    out = torch.empty(len(REDS), dtype=torch.int64, device="cuda")
    for i, op in enumerate(REDS):
        fks.fks_reduce_values(m, op, out=out[i:i + 1], stream=side)
    side.synchronize()
    got = to_np(out, "u64")
    assert [int(x) for x in got] == [ov.reduce_values(vals, op, 32) for op in REDS]


def test_reduce_after_map_at_2_24():
    """A larger map (2^24 keys): the sum after an add equals the oracle's fold of the mapped
    values, and the mapped table keeps every key word and header byte of the source."""
    fks = _fks()
    n = 1 << 24
    announce(f"gpu reduce after map: n={n}")
    keys = workloads.unique_u64(n, 2024, dense_fraction=0.5)
    vals = np.arange(n, dtype=np.uint32)
    m = fks.fks_build_u64(to_dev(keys), to_dev(vals), 0xABC)
    m2 = fks.fks_map_values(m, fks.FKS_VOP_AFFINE, 3, 1 << 31)
    mapped = ov.map_values(vals, ov.VOP_AFFINE, 3, 1 << 31)
    for op in REDS:
        assert fks.fks_reduce_values(m2, op) == ov.reduce_values(mapped, op, 32), op
    h, s, _ = fks.fks_export(m)
    h2, s2, _ = fks.fks_export(m2)
    assert (h == h2).all()
    c, c2 = s.reshape(-1, 16), s2.reshape(-1, 16)
    assert (c[:, 0:8] == c2[:, 0:8]).all() and (c[:, 12:16] == c2[:, 12:16]).all()
    old = c[:, 8:12].copy().view(np.uint32).ravel()
    new = c2[:, 8:12].copy().view(np.uint32).ravel()
    assert (new == ov.map_values(old, ov.VOP_AFFINE, 3, 1 << 31)).all()
