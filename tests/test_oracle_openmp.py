"""The OpenMP build of the oracle (the all-cores leg of the CPU baseline) gives the bytes and
answers of the sequential oracle: its parallel loops are independent per key, bucket, group
or query, so the table is the same whatever the thread count."""
import numpy as np
import pytest

import oracle
from oracle import cbind
from paper_2508_11443_amd import workloads
from tests import collide


@pytest.mark.parametrize("n,sigma", [(0, 1), (1, 2), (1000, 3), ((1 << 18) + 77, 0xF00D)])
def test_openmp_u64_equals_sequential(n, sigma):
    keys = workloads.unique_u64(n, n + 9, dense_fraction=0.5)
    vals = np.arange(n, dtype=np.uint32)
    a = oracle.build_u64(keys, vals, sigma)
    b = oracle.build_u64(keys, vals, sigma, omp=True)
    assert a.info == b.info
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    q, _ = workloads.u64_queries(keys, 2 * n + 10, 0.5, 4)
    for x, y in zip(a.lookup(q), b.lookup(q)):
        assert np.array_equal(x, y)


def test_openmp_rejections_and_errors_equal_sequential():
    # forced level-one rejections (c = 1) and a repeated key take the same paths
    keys = workloads.unique_u64(5000, 21)
    vals = np.arange(5000, dtype=np.uint32)
    a = oracle.build_u64(keys, vals, 7, c=2, T=8)
    b = oracle.build_u64(keys, vals, 7, c=2, T=8, omp=True)
    assert a.info == b.info and all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    dup = np.concatenate([keys, keys[:1]])
    for omp in (False, True):
        with pytest.raises(oracle.OracleError) as e:
            oracle.build_u64(dup, np.zeros(dup.size, np.uint32), 7, omp=omp)
        assert e.value.code == oracle.EDUPKEY


def test_openmp_strings_with_a_fingerprint_collision():
    off, data, _, _ = collide.strings_with_collision(0xC0111DE, 3000, 77)
    vals = np.arange(off.size - 1, dtype=np.uint32)
    a = oracle.build_bytes(off, data, vals, 0xC0111DE)
    b = oracle.build_bytes(off, data, vals, 0xC0111DE, omp=True)
    assert a.info == b.info and a.r == 1
    assert all(np.array_equal(x, y) for x, y in zip(a.export(), b.export()))
    for x, y in zip(a.lookup_bytes(off, data), b.lookup_bytes(off, data)):
        assert np.array_equal(x, y)


def test_thread_counts():
    assert cbind.threads(False) == 1
    assert cbind.threads(True) >= 1
