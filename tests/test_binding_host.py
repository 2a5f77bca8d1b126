"""Host-side checks of the Python binding, before any device work: an output tensor shorter than
the needle count (or a map-id array shorter than the needles) is refused with ValueError, since
the kernels write one entry per needle; a host tensor where a device buffer is due is a
TypeError.  No call here reaches a kernel."""
import pytest

torch = pytest.importorskip("torch")


def _fks():
    from paper_2508_11443_amd import fks
    return fks


def _i64(n):
    return torch.zeros(n, dtype=torch.int64)


def _i32(n):
    return torch.zeros(n, dtype=torch.int32)


def _u8(n):
    return torch.zeros(n, dtype=torch.uint8)


def test_short_outputs_are_refused():
    fks = _fks()
    m = fks.FksMap(0, "u64")
    q = _i64(10)
    short = [
        lambda: fks.fks_lookup_u64(m, q, _i32(9), _u8(10)),
        lambda: fks.fks_lookup_u64(m, q, _i32(10), _u8(9)),
        lambda: fks.fks_contains_u64(m, q, _u8(0)),
        lambda: fks.fks_lookup_u64_v64(m, q, _i64(9)),
        lambda: fks.fks_lookup_bytes(m, _i64(11), _u8(4), _i32(9), None),
        lambda: fks.fks_contains_bytes(m, _i64(11), _u8(4), _u8(9)),
        lambda: fks.fks_sorted_lookup_u64(fks.FksSorted(0, 0), q, _i32(10), _u8(3)),
        lambda: fks.fks_reduce_values(m, fks.FKS_VRED_SUM, out=_i64(0)),
    ]
    for call in short:
        with pytest.raises(ValueError):
            call()


def test_batch_map_ids_must_cover_the_needles():
    fks = _fks()
    b = fks.FksBatch(0, 0)
    with pytest.raises(ValueError):
        fks.fks_lookup_batch_u64(b, _i32(5), _i64(10), _i32(10), _u8(10))


def test_sized_host_tensors_are_refused_as_host_memory():
    fks = _fks()
    m = fks.FksMap(0, "u64")
    with pytest.raises(TypeError):
        fks.fks_lookup_u64(m, _i64(10), _i32(10), _u8(10))
