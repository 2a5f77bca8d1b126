"""GPU test of fks_reduce_values_noalloc, the reduction for callers that cannot allocate:
through the C ABI, its fold equals fks_reduce_values' (and the oracle's fold over the input
values) on two calls in a row on one stream, the second over a smaller map, for every fold
operation and every kind of map; an empty map gives the identities."""
import numpy as np
import pytest

from oracle import values as ov
from paper_2508_11443_amd import workloads
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

REDS = [ov.VRED_SUM, ov.VRED_MIN, ov.VRED_MAX, ov.VRED_XOR]


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def _u32_map(n, seed):
    fks = _fks()
    keys = workloads.unique_u64(n, seed, dense_fraction=0.5)
    vals = np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return fks.fks_build_u64(to_dev(keys), to_dev(vals), seed + 1), vals, 32


def _u64_map(n, seed):
    fks = _fks()
    keys = workloads.unique_u64(n, seed, dense_fraction=0.5)
    vals = np.random.default_rng(seed).integers(0, 1 << 64, size=n, dtype=np.uint64)
    return fks.fks_build_u64_v64(to_dev(keys), to_dev(vals), seed + 1), vals, 64


def _bytes_map(n, seed):
    fks = _fks()
    off, data = workloads.random_strings(n, seed, 4, 64)
    vals = np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return fks.fks_build_bytes(to_dev(off), to_dev(data), to_dev(vals), seed + 1), vals, 32


@pytest.mark.parametrize("make,big,small", [(_u32_map, (1 << 22) + 77, 1000), (_u64_map, 300007, 9),
                                            (_bytes_map, 200003, 33)])
def test_noalloc_reduce_equals_reduce_twice(make, big, small):
    import torch
    fks = _fks()
    announce(f"gpu no-alloc reduce: {make.__name__} n={big} then n={small}")
    m1, v1, w = make(big, 11)
    m2, v2, _ = make(small, 12)
    dev = torch.device("cuda", torch.cuda.current_device())
    for op in REDS:
        out = torch.full((4,), -1, dtype=torch.int64, device=dev)
        fks.fks_reduce_values_noalloc(m1, op, out[0:1])
        fks.fks_reduce_values_noalloc(m2, op, out[1:2])
        fks.fks_reduce_values(m1, op, out=out[2:3])
        fks.fks_reduce_values(m2, op, out=out[3:4])
        torch.cuda.synchronize()
        got = [int(x) for x in out.cpu().numpy().view(np.uint64)]
        assert got[0] == got[2] == ov.reduce_values(v1, op, w), (make.__name__, op)
        assert got[1] == got[3] == ov.reduce_values(v2, op, w), (make.__name__, op)
    m1.destroy()
    m2.destroy()


def test_noalloc_reduce_empty_map():
    import torch
    fks = _fks()
    announce("gpu no-alloc reduce: empty map")
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    m = fks.fks_build_u64(e, torch.empty(0, dtype=torch.int32, device="cuda"), 3)
    for op in REDS:
        out = torch.full((2,), 7, dtype=torch.int64, device="cuda")
        fks.fks_reduce_values_noalloc(m, op, out[0:1])
        fks.fks_reduce_values(m, op, out=out[1:2])
        torch.cuda.synchronize()
        got = [int(x) for x in out.cpu().numpy().view(np.uint64)]
        assert got[0] == got[1] == ov.reduce_values(np.zeros(0, np.uint32), op, 32), op
    m.destroy()


def test_noalloc_reduce_rejects_bad_arguments():
    fks = _fks()
    lib = fks.library()
    assert lib.fks_reduce_values_noalloc(None, 0, None, None) == fks.FKS_EINVAL
