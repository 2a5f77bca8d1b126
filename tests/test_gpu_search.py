"""GPU parity of the comparison maps (sorted array + binary search, Eytzinger order;
Section 4) against the CPU oracle, through the C ABI.

The layouts are unique for distinct keys, so the exported key and value arrays
must equal the oracle's element by element; lookups must equal the oracle's
(dictionary semantics).  Sizes span one tile (4096 records), several workers of
the radix sort and ragged tails; keys include one dense run (long stretches of
equal high digits) and the extreme values 0 and 2^64 - 1."""
import numpy as np
import pytest

import oracle
from paper_2508_11443_amd import workloads
from tests import searchcheck
from tests.gpu_util import announce, empty, to_dev, to_np

pytestmark = pytest.mark.gpu

MISSING = 0xC0FFEE
SIZES = [1, 2, 3, 4, 5, 7, 8, 100, 4095, 4096, 4097, 40000, 65536 + 3, (1 << 20) + 77]


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def gpu_lookup(s, q):
    import torch
    v = empty(q.size, "u32")
    f = empty(q.size, "u8")
    _fks().fks_sorted_lookup_u64(s, to_dev(q), v, f, missing=MISSING)
    torch.cuda.synchronize()
    return to_np(v, "u32"), to_np(f, "u8")


def _queries(keys, m, seed):
    q, expect = workloads.u64_queries(keys, m, 0.5, seed)
    extra = np.concatenate([keys[:50] + np.uint64(1), keys[:50] - np.uint64(1),
                            np.array([0, 1, 2**64 - 1, 2**64 - 2], np.uint64)])
    return np.concatenate([q, extra])


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n", SIZES)
def test_layout_and_lookup_match_oracle(layout, n):
    announce(f"gpu search: layout={layout} n={n}")
    keys = workloads.unique_u64(n, 3 * n + layout, dense_fraction=0.5)
    vals = np.random.default_rng(n).integers(0, 2**32, size=n, dtype=np.uint32)
    s = _fks().fks_sorted_build_u64(to_dev(keys), to_dev(vals), layout)
    gk, gv = _fks().fks_sorted_export(s)
    rk, rv = oracle.search_build(keys, vals, layout)
    assert (gk == rk).all() and (gv == rv).all()
    q = _queries(keys, max(2 * n, 1000), n)
    v, f = gpu_lookup(s, q)
    ov, of = oracle.search_lookup(rk, rv, layout, q, missing=MISSING)
    assert (f == of).all() and (v == ov).all()


@pytest.mark.parametrize("layout", [0, 1])
def test_extremes_empty_and_duplicates(layout):
    fks = _fks()
    announce(f"gpu search: extremes layout={layout}")
    keys = np.array([2**64 - 1, 0, 1, 2**63, 2**32], np.uint64)
    vals = np.arange(5, dtype=np.uint32) + 10
    s = fks.fks_sorted_build_u64(to_dev(keys), to_dev(vals), layout)
    q = np.array([0, 1, 2, 2**64 - 1, 2**64 - 2, 2**63, 2**32, 2**32 - 1], np.uint64)
    v, f = gpu_lookup(s, q)
    assert f.tolist() == [1, 1, 0, 1, 0, 1, 1, 0]
    assert v.tolist() == [11, 12, MISSING, 10, MISSING, 13, 14, MISSING]
    # the empty map: every needle is absent
    e = fks.fks_sorted_build_u64(to_dev(keys[:0]), to_dev(vals[:0]), layout)
    v, f = gpu_lookup(e, q)
    assert not f.any() and (v == MISSING).all()
    # equal keys break the precondition
    dup = np.concatenate([workloads.unique_u64(9000, 1), np.array([0], np.uint64)])
    dup[-1] = dup[4321]
    with pytest.raises(fks.FksError) as err:
        fks.fks_sorted_build_u64(to_dev(dup), to_dev(np.zeros(dup.size, np.uint32)), layout)
    assert err.value.code == fks.FKS_EDUPKEY


@pytest.fixture(scope="module")
def bench_inputs():
    """The benchmark's 2^26 keys and needles, generated once for both layouts."""
    n = 1 << 26
    keys = workloads.unique_u64(n, 2026, dense_fraction=0.5)
    order = np.argsort(keys, kind="stable")
    q, expect, src = workloads.u64_queries(keys, n, 0.5, 2027, return_index=True)
    return keys, order, q, expect, src


@pytest.mark.parametrize("layout", [0, 1])
def test_bench_size(layout, bench_inputs):
    """2^26 keys (half uniform, half one dense run), as the benchmark builds them:
    the sorted layout must be the keys in increasing order with their values; the
    Eytzinger layout must be that array gathered in level order; 2^26 needles at
    50% hits against dictionary semantics."""
    import torch
    keys, order, q, expect, src = bench_inputs
    n = keys.size
    announce(f"gpu search: bench size layout={layout}")
    vals = np.arange(n, dtype=np.uint32)
    s = _fks().fks_sorted_build_u64(to_dev(keys), to_dev(vals), layout)
    gk, gv = _fks().fks_sorted_export(s)
    if layout == 0:
        assert (gk == keys[order]).all() and (gv == order.astype(np.uint32)).all()
    else:
        # level-order node i holds the sorted pair of rank inorder_rank(i): a sample
        # of nodes (the helper is pinned against the oracle's recursive fill)
        rng = np.random.default_rng(7)
        nodes = np.concatenate([np.arange(1, 64), rng.integers(1, n + 1, size=2000)])
        for i in nodes.tolist():
            r = searchcheck.inorder_rank(i, n)
            assert gk[i - 1] == keys[order[r]] and gv[i - 1] == order[r]
    v, f = gpu_lookup(s, q)
    assert (f == expect).all()
    hit = expect == 1
    assert (v[hit] == src[hit].astype(np.uint32)).all()
    assert (v[~hit] == MISSING).all()
    del s
    torch.cuda.empty_cache()
