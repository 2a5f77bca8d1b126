"""GPU tests of the fks_allocator hook: every build entry point takes its map and scratch
from the caller's allocator and returns all of it (a counting allocator balances after
release, and the tables equal those of the default pool), and an allocator that fails at
any one of a build's allocations makes the call return FKS_ENOMEM with nothing leaked and
the out-parameter untouched.  All calls go through the C ABI."""
import ctypes
import gc

import numpy as np
import pytest

import oracle
from paper_2508_11443_amd import workloads
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _fks():
    from paper_2508_11443_amd import fks
    return fks


class Counting:
    """torch's caching allocator underneath; counts live blocks; optionally fails the k-th
    allocation (1-based) of its life."""

    def __init__(self, fail_at=0):
        import torch
        self.dev = torch.cuda.current_device()
        self.live = {}
        self.allocs = 0
        self.frees = 0
        self.fail_at = fail_at
        fks = _fks()
        self.alloc_obj = fks.Allocator(self._alloc, self._free)

    def _alloc(self, nbytes, stream):
        import torch
        self.allocs += 1
        if self.fail_at and self.allocs == self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, self.dev, stream)
        self.live[p] = nbytes
        return p

    def _free(self, ptr, stream):
        import torch
        assert ptr in self.live, "freed a pointer this allocator did not hand out"
        del self.live[ptr]
        self.frees += 1
        torch.cuda.caching_allocator_delete(ptr)


def _builders():
    """(name, build(allocator) -> object with destroy(), bytes of the table or None)."""
    import torch
    fks = _fks()
    keys = workloads.unique_u64(20000, 31, dense_fraction=0.5)
    vals = np.arange(20000, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    dv64 = to_dev(vals.astype(np.uint64) << np.uint64(33))
    off, data = workloads.random_strings(3000, 32, 4, 64)
    doff, ddata, dsv = to_dev(off), to_dev(data), to_dev(np.arange(3000, dtype=np.uint32))
    rep = to_dev(np.repeat(keys[:5000], 2))
    repv = to_dev(np.arange(10000, dtype=np.uint32))
    boff = np.array([0, 3000, 12000, 20000], np.uint64)
    base = fks.fks_build_u64(dk, dv, 5)
    return [
        ("u64", lambda a: fks.fks_build_u64(dk, dv, 5, allocator=a), fks.fks_export),
        ("u64 rounds", lambda a: fks.fks_build_u64(dk, dv, 5, schedule=1, allocator=a), fks.fks_export),
        ("u64_v64", lambda a: fks.fks_build_u64_v64(dk, dv64, 5, allocator=a), fks.fks_export),
        ("bytes", lambda a: fks.fks_build_bytes(doff, ddata, dsv, 5, allocator=a), fks.fks_export),
        ("from_array", lambda a: fks.fks_build_u64_from_array(rep, repv, 5, allocator=a), fks.fks_export),
        ("map_values", lambda a: fks.fks_map_values(base, fks.FKS_VOP_ADD, 7, allocator=a), fks.fks_export),
        ("batch", lambda a: fks.fks_build_batch_u64(dk, dv, boff, 9, allocator=a),
         lambda b: fks.fks_batch_export(b, 1)[:2]),
        ("sorted", lambda a: fks.fks_sorted_build_u64(dk, dv, fks.FKS_LAYOUT_EYTZINGER, allocator=a),
         fks.fks_sorted_export),
    ], base, torch


def test_counting_allocator_balances_and_tables_match():
    builders, base, torch = _builders()
    for name, build, export in builders:
        announce(f"gpu alloc: counting allocator, {name}")
        ref = build(None)
        want = export(ref)
        ref.destroy()
        cnt = Counting()
        obj = build(cnt.alloc_obj)
        torch.cuda.synchronize()
        assert cnt.allocs >= 1 and cnt.live, name          # the object's memory is held
        got = export(obj)
        for a, b in zip(want, got):
            assert np.array_equal(a, b), name
        obj.destroy()
        torch.cuda.synchronize()
        assert not cnt.live and cnt.frees == cnt.allocs, name
    base.destroy()


def test_failing_allocator_returns_enomem_and_leaks_nothing():
    fks = _fks()
    builders, base, torch = _builders()
    for name, build, _ in builders:
        announce(f"gpu alloc: failing allocator, {name}")
        total = Counting()
        build(total.alloc_obj).destroy()
        assert total.allocs >= 1
        for k in range(1, total.allocs + 1):
            cnt = Counting(fail_at=k)
            with pytest.raises(fks.FksError) as e:
                build(cnt.alloc_obj)
            assert e.value.code == fks.FKS_ENOMEM, (name, k)
            torch.cuda.synchronize()
            assert not cnt.live, (name, k, cnt.live)
    base.destroy()


def test_failing_allocator_leaves_out_untouched():
    """Through the raw C ABI: *out keeps its previous value when the first allocation fails."""
    import torch
    fks = _fks()
    lib = fks.library()
    announce("gpu alloc: out-parameter untouched on FKS_ENOMEM")
    keys = to_dev(workloads.unique_u64(1000, 3))
    vals = to_dev(np.arange(1000, dtype=np.uint32))
    cnt = Counting(fail_at=1)
    out = ctypes.c_void_p(12345)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.fks_build_u64(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), 1000, 1, None,
                           cnt.alloc_obj.pointer(), stream, ctypes.byref(out))
    assert rc == fks.FKS_ENOMEM and out.value == 12345 and not cnt.live


def test_torch_allocator_holds_the_map():
    """The torch-backed allocator: torch sees the map's memory while it lives."""
    import torch
    fks = _fks()
    announce("gpu alloc: torch caching allocator")
    keys = workloads.unique_u64(1 << 20, 4)
    vals = np.arange(1 << 20, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    ref = oracle.build_u64(keys, vals, 3)
    rh, rs = ref.export()
    # Tensors of earlier tests can sit in reference cycles (exception tracebacks hold their
    # frames); collect them now and keep the collector off while torch's count is compared.
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        m = fks.fks_build_u64(dk, dv, 3, allocator=fks.torch_allocator())
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        assert held >= m.info()["device_bytes"]
        h, s, _ = fks.fks_export(m)
        assert (h == rh).all() and (s == rs).all()
        m.destroy()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    finally:
        gc.enable()
