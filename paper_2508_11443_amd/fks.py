"""Thin Python binding of ``libfks.so`` (the C ABI declared in include/fks.h).

Argument marshalling only: every step of a build or a lookup runs in the HIP
kernels of the library.  Device buffers are torch tensors on a ROCm device
(torch supplies the memory and the stream); the functions carry the names of
the C entry points they call.  There is no fallback: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfks.so")

FKS_OK, FKS_EINVAL, FKS_ENOMEM, FKS_EDUPKEY, FKS_EBUILD, FKS_EHIP = 0, -1, -2, -3, -4, -5
FKS_LAYOUT_SORTED, FKS_LAYOUT_EYTZINGER = 0, 1
FKS_VOP_ADD, FKS_VOP_MUL, FKS_VOP_XOR, FKS_VOP_AFFINE, FKS_VOP_GATHER = 0, 1, 2, 3, 4
FKS_VRED_SUM, FKS_VRED_MIN, FKS_VRED_MAX, FKS_VRED_XOR = 0, 1, 2, 3


class FksError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        lib = _load()
        msg = lib.fks_strerror(code).decode()
        if code == FKS_EHIP:
            msg += f" (hipError {lib.fks_last_hip_error()})"
        super().__init__(f"{what}: {msg}" if what else msg)
        self.code = code


class fks_params(ctypes.Structure):
    _fields_ = [("c", ctypes.c_uint32), ("T", ctypes.c_uint32), ("R", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32)]


class fks_prof_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class fks_map_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("S", ctypes.c_uint64), ("header_bytes", ctypes.c_uint64),
                ("slot_bytes", ctypes.c_uint64), ("ctx_bytes", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("r", ctypes.c_uint32), ("kind", ctypes.c_uint32),
                ("c", ctypes.c_uint32), ("T", ctypes.c_uint32), ("R", ctypes.c_uint32),
                ("max_t", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("size_hist", ctypes.c_uint64 * 16)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class fks_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class Allocator:
    """An fks_allocator backed by two Python callables: alloc(nbytes, stream) -> device address
    or 0, free(address, stream).  The object must outlive every map built with it (the map
    returns its memory through it in fks_destroy); the binding's map objects keep a reference."""

    def __init__(self, alloc, free):
        def _alloc(nbytes, stream, user):
            try:
                return alloc(int(nbytes), stream or 0) or None
            except Exception:
                return None

        def _free(ptr, stream, user):
            free(int(ptr), stream or 0)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = fks_allocator(self._alloc_cb, self._free_cb, None)

    def pointer(self):
        return ctypes.byref(self.struct)


def torch_allocator(device=None) -> Allocator:
    """Device memory from torch's caching allocator (torch.cuda.caching_allocator_alloc on
    the stream the library names, caching_allocator_delete to release), so that a map's
    memory is visible to, and reused by, the allocator the rest of the program uses.  Each
    allocation is a call from C back into Python (a few microseconds), so builds that
    allocate little and often may prefer the default (allocator=None: the device's
    stream-ordered pool)."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, dev, stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return Allocator(alloc, free)


def fks_reduce_values_noalloc(m: FksMap, op: int, out, stream=None):
    """fks_reduce_values into out (a one-element int64/uint64 device tensor) without any
    allocation: the library's static per-device scratch holds the partial folds.  Calls
    that overlap on one device race for that scratch.  Asynchronous; returns out."""
    _fits(1, out=out)
    rc = _load().fks_reduce_values_noalloc(m.handle, op, _dev(out, _u64_types(), "out"), _stream(stream))
    _check(rc, "fks_reduce_values_noalloc")
    return out


def _alloc_arg(allocator):
    return None if allocator is None else allocator.pointer()


_lib = None

# (name, restype, argtypes) of every exported entry point
_VP, _U64, _U32, _I32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
SIGNATURES = [
    ("fks_params_default", None, [_VP]),
    ("fks_build_u64", _I32, [_VP, _VP, _U64, _U64, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_build_u64_from_array", _I32, [_VP, _VP, _U64, _U64, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_build_u64_v64", _I32, [_VP, _VP, _U64, _U64, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_lookup_u64_v64", _I32, [_VP, _VP, _U64, _VP, _VP, _U64, _VP]),
    ("fks_build_bytes", _I32, [_VP, _VP, _U64, _VP, _U64, _U64, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_lookup_u64", _I32, [_VP, _VP, _U64, _VP, _VP, _U32, _VP]),
    ("fks_contains_u64", _I32, [_VP, _VP, _U64, _VP, _VP]),
    ("fks_lookup_bytes", _I32, [_VP, _VP, _VP, _U64, _U64, _VP, _VP, _U32, _VP]),
    ("fks_contains_bytes", _I32, [_VP, _VP, _VP, _U64, _U64, _VP, _VP]),
    ("fks_info", _I32, [_VP, _VP]),
    ("fks_map_values", _I32, [_VP, _U32, _U64, _U64, _VP, _U64, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_reduce_values", _I32, [_VP, _U32, _VP, _VP]),
    ("fks_reduce_values_noalloc", _I32, [_VP, _U32, _VP, _VP]),
    ("fks_export", _I32, [_VP, _VP, _VP, _VP]),
    ("fks_destroy", None, [_VP]),
    ("fks_strerror", ctypes.c_char_p, [_I32]),
    ("fks_last_hip_error", _I32, []),
    ("fks_version", _I32, []),
    ("fks_build_batch_u64", _I32, [_VP, _VP, _VP, _U32, _U64, _VP, _U32, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_lookup_batch_u64", _I32, [_VP, _VP, _VP, _U64, _VP, _VP, _U32, _VP]),
    ("fks_batch_status", _I32, [_VP, _VP, _VP, _VP]),
    ("fks_batch_info", _I32, [_VP, _U32, _VP]),
    ("fks_batch_export", _I32, [_VP, _U32, _VP, _VP, _VP]),
    ("fks_batch_destroy", None, [_VP]),
    ("fks_batch_set_schedule", _I32, [_U32, _U64, _U32]),
    ("fks_batch_schedules", _I32, [_VP, _I32]),
    ("fks_server_create", _I32, [_U64, _VP, _U32, ctypes.POINTER(_VP)]),
    ("fks_server_submit_build", _I32, [_VP, _VP, _VP, _U64, _U64, _VP, _VP, _VP]),
    ("fks_server_submit_lookup", _I32, [_VP, _U32, _VP, _U64, _VP, _VP, _U32, _VP, _VP]),
    ("fks_server_poll", _I32, [_VP, _U64, _VP, _VP, _VP]),
    ("fks_server_wait_all", _I32, [_VP]),
    ("fks_server_latencies", _I32, [_VP, _VP, _VP, _VP, _VP, _U64]),
    ("fks_server_stats", _I32, [_VP, _VP]),
    ("fks_server_map", _VP, [_VP, _U32]),
    ("fks_server_destroy", None, [_VP]),
    ("fks_probe_random_reads", _I32, [_U64, _U64, _U32, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("fks_sorted_build_u64", _I32, [_VP, _VP, _U64, _U32, _VP, _VP, ctypes.POINTER(_VP)]),
    ("fks_sorted_lookup_u64", _I32, [_VP, _VP, _U64, _VP, _VP, _U32, _VP]),
    ("fks_sorted_export", _I32, [_VP, _VP, _VP]),
    ("fks_sorted_info", _I32, [_VP, _VP, _VP]),
    ("fks_sorted_destroy", None, [_VP]),
    ("fks_prof_enable", _I32, [_I32]),
    ("fks_prof_reset", None, []),
    ("fks_prof_read", _I32, [_VP, _I32]),
]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _load()


def _check(rc: int, what: str):
    if rc != FKS_OK:
        raise FksError(rc, what)


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtypes, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _fits(count: int, **tensors):
    """Refuse, before any device work, a tensor that holds fewer than `count` entries where the
    call reads or writes one entry per needle (the kernels index it up to count)."""
    for name, t in tensors.items():
        if t is not None and t.numel() < count:
            raise ValueError(f"{name} holds {t.numel()} entries; the call touches {count}")


def _u64_types():
    import torch
    return (torch.int64, torch.uint64)


def _u32_types():
    import torch
    return (torch.int32, torch.uint32)


def _params(c=None, T=None, R=None, schedule=None):
    p = fks_params()
    _load().fks_params_default(ctypes.byref(p))
    if schedule is not None:
        p.schedule = schedule
    if c is not None:
        p.c = c
    if T is not None:
        p.T = T
    if R is not None:
        p.R = R
    return p


def _info_dict(inf) -> dict:
    d = {name: getattr(inf, name) for name, _ in fks_map_info._fields_}
    d["size_hist"] = [int(x) for x in inf.size_hist]
    return d


class FksMap:
    """A built map; owns the C handle and releases it with fks_destroy (through the allocator
    it was built with, which the object keeps alive)."""

    def __init__(self, handle: int, kind: str, allocator=None):
        self._h = ctypes.c_void_p(handle)
        self.kind = kind
        self._allocator = allocator

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = fks_map_info()
        _check(_load().fks_info(self._h, ctypes.byref(inf)), "fks_info")
        return _info_dict(inf)

    def destroy(self):
        if self._h is not None and self._h.value:
            _load().fks_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fks_build_u64(keys, vals, seed: int, c=None, T=None, R=None, stream=None, schedule=None,
                  allocator=None) -> FksMap:
    """from_array_nodup over n uint64 keys (device tensor, int64 or uint64) and uint32 values.
    schedule=1 searches level two with the paper's flattened rounds (same table).
    allocator: an Allocator (e.g. torch_allocator()) for the map and the build's scratch, or
    None for the device's stream-ordered pool."""
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    p = _params(c, T, R, schedule)
    out = ctypes.c_void_p()
    rc = _load().fks_build_u64(_dev(keys, _u64_types(), "keys"), _dev(vals, _u32_types(), "vals"), n,
                               seed & ((1 << 64) - 1), ctypes.byref(p), _alloc_arg(allocator), _stream(stream),
                               ctypes.byref(out))
    _check(rc, "fks_build_u64")
    return FksMap(out.value, "u64", allocator)


def fks_build_u64_from_array(keys, vals, seed: int, c=None, T=None, R=None, stream=None,
                             allocator=None) -> FksMap:
    """from_array: keys may repeat; a repeated key keeps the value of its first occurrence."""
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    p = _params(c, T, R)
    out = ctypes.c_void_p()
    rc = _load().fks_build_u64_from_array(_dev(keys, _u64_types(), "keys"), _dev(vals, _u32_types(), "vals"), n,
                                          seed & ((1 << 64) - 1), ctypes.byref(p), _alloc_arg(allocator),
                                          _stream(stream), ctypes.byref(out))
    _check(rc, "fks_build_u64_from_array")
    return FksMap(out.value, "u64", allocator)


def fks_build_u64_v64(keys, vals, seed: int, c=None, T=None, R=None, stream=None, allocator=None) -> FksMap:
    """from_array_nodup with 64-bit values (device tensor, int64 or uint64)."""
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    p = _params(c, T, R)
    out = ctypes.c_void_p()
    rc = _load().fks_build_u64_v64(_dev(keys, _u64_types(), "keys"), _dev(vals, _u64_types(), "vals"), n,
                                   seed & ((1 << 64) - 1), ctypes.byref(p), _alloc_arg(allocator),
                                   _stream(stream), ctypes.byref(out))
    _check(rc, "fks_build_u64_v64")
    return FksMap(out.value, "u64v64", allocator)


def fks_map_values(m: FksMap, op: int, a: int = 0, b: int = 0, table=None, stream=None,
                   allocator=None) -> FksMap:
    """A new map with the keys of m and op(v) as values (FKS_VOP_*); table: the device tensor
    FKS_VOP_GATHER reads (uint32 entries, or 64-bit for maps with 64-bit values)."""
    if table is not None:
        kinds = _u64_types() if m.kind == "u64v64" else _u32_types()
        d_table, n_table = _dev(table, kinds, "table"), table.numel()
    else:
        d_table, n_table = None, 0
    out = ctypes.c_void_p()
    mask = (1 << 64) - 1
    rc = _load().fks_map_values(m.handle, op, a & mask, b & mask, d_table, n_table, _alloc_arg(allocator),
                                _stream(stream), ctypes.byref(out))
    _check(rc, "fks_map_values")
    return FksMap(out.value, m.kind, allocator)


def fks_reduce_values(m: FksMap, op: int, out=None, stream=None):
    """Fold of op (FKS_VRED_*) over the map's values, each key once.  With out (a one-element
    int64/uint64 device tensor) the call is asynchronous and returns out; without it, the
    result is returned as a Python int."""
    import torch
    _fits(1, out=out)
    own = out is None
    if own:
        out = torch.empty(1, dtype=torch.int64, device=torch.device("cuda", torch.cuda.current_device()))
    rc = _load().fks_reduce_values(m.handle, op, _dev(out, _u64_types(), "out"), _stream(stream))
    _check(rc, "fks_reduce_values")
    if not own:
        return out
    torch.cuda.synchronize()   # the fold may run on a stream other than the current one
    return int(out.cpu().numpy().view("uint64")[0])


def fks_lookup_u64_v64(m: FksMap, queries, vals_out, found_out=None, missing: int = 2**64 - 1, stream=None):
    import torch
    _fits(queries.numel(), vals_out=vals_out, found_out=found_out)
    rc = _load().fks_lookup_u64_v64(m.handle, _dev(queries, _u64_types(), "queries"), queries.numel(),
                                    _dev(vals_out, _u64_types(), "vals_out"),
                                    _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                    missing & ((1 << 64) - 1), _stream(stream))
    _check(rc, "fks_lookup_u64_v64")


def fks_build_bytes(offsets, data, vals, seed: int, c=None, T=None, R=None, stream=None,
                    allocator=None) -> FksMap:
    """from_array_nodup over n byte-string keys given as CSR (int64 offsets[n+1], uint8 bytes)."""
    import torch
    n = offsets.numel() - 1
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    p = _params(c, T, R)
    out = ctypes.c_void_p()
    rc = _load().fks_build_bytes(_dev(offsets, (torch.int64,), "offsets"),
                                 _dev(data, (torch.uint8,), "bytes") if data.numel() else None,
                                 data.numel(), _dev(vals, _u32_types(), "vals"), n,
                                 seed & ((1 << 64) - 1), ctypes.byref(p), _alloc_arg(allocator),
                                 _stream(stream), ctypes.byref(out))
    _check(rc, "fks_build_bytes")
    return FksMap(out.value, "bytes", allocator)


def fks_lookup_u64(m: FksMap, queries, vals_out, found_out, missing: int = 0xFFFFFFFF, stream=None):
    import torch
    _fits(queries.numel(), vals_out=vals_out, found_out=found_out)
    rc = _load().fks_lookup_u64(m.handle, _dev(queries, _u64_types(), "queries"), queries.numel(),
                                _dev(vals_out, _u32_types(), "vals_out"),
                                _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                missing & 0xFFFFFFFF, _stream(stream))
    _check(rc, "fks_lookup_u64")


def fks_contains_u64(m: FksMap, queries, found_out, stream=None):
    import torch
    _fits(queries.numel(), found_out=found_out)
    rc = _load().fks_contains_u64(m.handle, _dev(queries, _u64_types(), "queries"), queries.numel(),
                                  _dev(found_out, (torch.uint8, torch.bool), "found_out"), _stream(stream))
    _check(rc, "fks_contains_u64")


def fks_lookup_bytes(m: FksMap, q_offsets, q_data, vals_out, found_out, missing: int = 0xFFFFFFFF,
                     stream=None):
    import torch
    _fits(q_offsets.numel() - 1, vals_out=vals_out, found_out=found_out)
    rc = _load().fks_lookup_bytes(m.handle, _dev(q_offsets, (torch.int64,), "q_offsets"),
                                  _dev(q_data, (torch.uint8,), "q_bytes") if q_data.numel() else None,
                                  q_data.numel(), q_offsets.numel() - 1, _dev(vals_out, _u32_types(), "vals_out"),
                                  _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                  missing & 0xFFFFFFFF, _stream(stream))
    _check(rc, "fks_lookup_bytes")


def fks_contains_bytes(m: FksMap, q_offsets, q_data, found_out, stream=None):
    import torch
    _fits(q_offsets.numel() - 1, found_out=found_out)
    rc = _load().fks_contains_bytes(m.handle, _dev(q_offsets, (torch.int64,), "q_offsets"),
                                    _dev(q_data, (torch.uint8,), "q_bytes") if q_data.numel() else None,
                                    q_data.numel(), q_offsets.numel() - 1,
                                    _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                    _stream(stream))
    _check(rc, "fks_contains_bytes")


def fks_info(m: FksMap) -> dict:
    return m.info()


def fks_export(m: FksMap):
    """Host copies (header uint8[], cells uint8[], level-two triples uint64[T,3]) of a map."""
    import numpy as np
    inf = m.info()
    header = np.zeros(inf["header_bytes"], np.uint8)
    slots = np.zeros(inf["slot_bytes"], np.uint8)
    consts = np.zeros((inf["T"], 3), np.uint64)
    rc = _load().fks_export(m.handle, header.ctypes.data if header.size else None,
                            slots.ctypes.data if slots.size else None, consts.ctypes.data)
    _check(rc, "fks_export")
    return header, slots, consts


def fks_destroy(m: FksMap):
    m.destroy()


def fks_version() -> int:
    return _load().fks_version()


def fks_prof_enable(on: bool = True):
    _load().fks_prof_enable(1 if on else 0)


def fks_prof_reset():
    _load().fks_prof_reset()


def fks_prof_read() -> dict:
    """{kernel name: (launches, total ms)} of the launches timed since the last reset."""
    lib = _load()
    cnt = lib.fks_prof_read(None, 0)
    arr = (fks_prof_entry * max(cnt, 1))()
    got = lib.fks_prof_read(ctypes.cast(arr, ctypes.c_void_p), cnt)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(got)}


# ---- batches of maps -------------------------------------------------------------

class FksBatch:
    """M independent maps built in one persistent launch; owns the C handle."""

    def __init__(self, handle: int, M: int, allocator=None):
        self._h = ctypes.c_void_p(handle)
        self.M = M
        self._allocator = allocator

    @property
    def handle(self):
        return self._h

    def status(self):
        import numpy as np
        st = np.zeros(self.M, np.int32)
        r = np.zeros(self.M, np.uint32)
        S = np.zeros(self.M, np.uint32)
        _check(_load().fks_batch_status(self._h, st.ctypes.data, r.ctypes.data, S.ctypes.data),
               "fks_batch_status")
        return st, r, S

    def destroy(self):
        if self._h is not None and self._h.value:
            _load().fks_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fks_build_batch_u64(keys, vals, map_offsets, batch_seed: int, c=None, T=None, R=None, schedule: int = 0,
                        stream=None, allocator=None) -> FksBatch:
    """Build M maps: map m holds keys[map_offsets[m]:map_offsets[m+1]] (host offsets, M+1 entries)."""
    import numpy as np
    off = np.ascontiguousarray(map_offsets, np.uint64)
    M = off.size - 1
    p = _params(c, T, R)
    out = ctypes.c_void_p()
    rc = _load().fks_build_batch_u64(_dev(keys, _u64_types(), "keys") if keys.numel() else None,
                                     _dev(vals, _u32_types(), "vals") if vals.numel() else None,
                                     off.ctypes.data, M, batch_seed & ((1 << 64) - 1), ctypes.byref(p),
                                     schedule, _alloc_arg(allocator), _stream(stream), ctypes.byref(out))
    _check(rc, "fks_build_batch_u64")
    return FksBatch(out.value, M, allocator)


def fks_lookup_batch_u64(b: FksBatch, map_ids, queries, vals_out, found_out, missing: int = 0xFFFFFFFF,
                         stream=None):
    import torch
    _fits(queries.numel(), map_ids=map_ids, vals_out=vals_out, found_out=found_out)
    rc = _load().fks_lookup_batch_u64(b.handle, _dev(map_ids, _u32_types(), "map_ids"),
                                      _dev(queries, _u64_types(), "queries"), queries.numel(),
                                      _dev(vals_out, _u32_types(), "vals_out"),
                                      _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                      missing & 0xFFFFFFFF, _stream(stream))
    _check(rc, "fks_lookup_batch_u64")


def fks_batch_export(b: FksBatch, index: int):
    """(header, cells, level-two triples) of map `index` of a batch, as host arrays."""
    import numpy as np
    inf = fks_map_info()
    rc = _load().fks_batch_info(b.handle, index, ctypes.byref(inf))
    _check(rc, "fks_batch_info")
    header = np.zeros(inf.header_bytes, np.uint8)
    slots = np.zeros(inf.slot_bytes, np.uint8)
    consts = np.zeros((inf.T, 3), np.uint64)
    rc = _load().fks_batch_export(b.handle, index, header.ctypes.data if header.size else None,
                                  slots.ctypes.data if slots.size else None, consts.ctypes.data)
    _check(rc, "fks_batch_export")
    return header, slots, consts, _info_dict(inf)


def fks_batch_schedules():
    import numpy as np
    lib = _load()
    cnt = lib.fks_batch_schedules(None, 0)
    out = np.zeros(cnt, np.uint32)
    lib.fks_batch_schedules(out.ctypes.data, cnt)
    return [int(x) for x in out]


def fks_batch_set_schedule(M: int, total_keys: int, schedule: int):
    _check(_load().fks_batch_set_schedule(M, total_keys, schedule), "fks_batch_set_schedule")


def fks_batch_destroy(b: FksBatch):
    b.destroy()


# ---- serving -----------------------------------------------------------------------

class fks_server_stats_t(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("lookup_launches", ctypes.c_uint64), ("graph_replays", ctypes.c_uint64),
                ("graphs_captured", ctypes.c_uint64), ("coalesced_requests", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("queries_done", ctypes.c_uint64), ("keys_built", ctypes.c_uint64),
                ("span_ms", ctypes.c_double), ("resident_maps", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class FksServer:
    """fks_server_*: resident maps, budgeted builds, coalesced graph-replayed lookups.
    Keeps a reference to every tensor handed to a request until the server is waited on."""

    def __init__(self, budget_bytes: int, c=None, T=None, R=None, graphs: bool = True):
        p = _params(c, T, R)
        out = ctypes.c_void_p()
        _check(_load().fks_server_create(budget_bytes, ctypes.byref(p), 0 if graphs else 1, ctypes.byref(out)),
               "fks_server_create")
        self._h = out
        self._keep = {}

    def submit_build(self, keys, vals, seed: int, stream=None):
        """Queue a build; its device work is ordered after everything already queued on
        `stream` (default: torch's current stream), so the keys may still be in flight."""
        rid, mid = ctypes.c_uint64(), ctypes.c_uint32()
        _check(_load().fks_server_submit_build(self._h, _dev(keys, _u64_types(), "keys"),
                                               _dev(vals, _u32_types(), "vals"), keys.numel(),
                                               seed & ((1 << 64) - 1), _stream(stream), ctypes.byref(rid),
                                               ctypes.byref(mid)),
               "fks_server_submit_build")
        self._keep[rid.value] = (keys, vals)
        return rid.value, mid.value

    def submit_lookup(self, map_id: int, queries, vals_out, found_out, missing: int = 0xFFFFFFFF, stream=None):
        """Queue a lookup, ordered after `stream` as submit_build is."""
        import torch
        _fits(queries.numel(), vals_out=vals_out, found_out=found_out)
        rid = ctypes.c_uint64()
        _check(_load().fks_server_submit_lookup(self._h, map_id, _dev(queries, _u64_types(), "queries"),
                                                queries.numel(), _dev(vals_out, _u32_types(), "vals_out"),
                                                _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                                missing & 0xFFFFFFFF, _stream(stream), ctypes.byref(rid)),
               "fks_server_submit_lookup")
        self._keep[rid.value] = (queries, vals_out, found_out)
        return rid.value

    def poll(self, rid: int):
        done, status, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(_load().fks_server_poll(self._h, rid, ctypes.byref(done), ctypes.byref(status), ctypes.byref(lat)),
               "fks_server_poll")
        return bool(done.value), status.value, lat.value

    def wait_all(self):
        _check(_load().fks_server_wait_all(self._h), "fks_server_wait_all")
        self._keep.clear()

    def latencies(self, count: int):
        import numpy as np
        sub = np.zeros(count, np.float64)
        done = np.zeros(count, np.float64)
        kind = np.zeros(count, np.int32)
        st = np.zeros(count, np.int32)
        got = _load().fks_server_latencies(self._h, sub.ctypes.data, done.ctypes.data, kind.ctypes.data,
                                           st.ctypes.data, count)
        return sub[:got], done[:got], kind[:got], st[:got]

    def stats(self) -> dict:
        st = fks_server_stats_t()
        _check(_load().fks_server_stats(self._h, ctypes.byref(st)), "fks_server_stats")
        return {name: getattr(st, name) for name, _ in fks_server_stats_t._fields_}

    def map_handle(self, map_id: int):
        return _load().fks_server_map(self._h, map_id)

    def destroy(self):
        if self._h is not None and self._h.value:
            _load().fks_server_destroy(self._h)
        self._h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fks_probe_random_reads(buffer_bytes: int = 2 << 30, probes: int = 1 << 27, width_bytes: int = 16,
                           stream=None) -> float:
    """Milliseconds for `probes` random reads of `width_bytes` from a buffer of `buffer_bytes`."""
    ms = ctypes.c_double()
    _check(_load().fks_probe_random_reads(buffer_bytes, probes, width_bytes, _stream(stream), ctypes.byref(ms)),
           "fks_probe_random_reads")
    return ms.value


# ---- comparison maps: sorted array / Eytzinger order -------------------------

class FksSorted:
    """A sorted-array or Eytzinger-layout map; released with fks_sorted_destroy."""

    def __init__(self, handle: int, layout: int, allocator=None):
        self._h = ctypes.c_void_p(handle)
        self.layout = layout
        self._allocator = allocator

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, layout = ctypes.c_uint64(), ctypes.c_uint32()
        _check(_load().fks_sorted_info(self._h, ctypes.byref(n), ctypes.byref(layout)), "fks_sorted_info")
        return {"n": n.value, "layout": layout.value}

    def destroy(self):
        if self._h is not None and self._h.value:
            _load().fks_sorted_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fks_sorted_build_u64(keys, vals, layout: int = FKS_LAYOUT_SORTED, stream=None, allocator=None) -> FksSorted:
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    out = ctypes.c_void_p()
    rc = _load().fks_sorted_build_u64(_dev(keys, _u64_types(), "keys"), _dev(vals, _u32_types(), "vals"), n,
                                      layout, _alloc_arg(allocator), _stream(stream), ctypes.byref(out))
    _check(rc, "fks_sorted_build_u64")
    return FksSorted(out.value, layout, allocator)


def fks_sorted_lookup_u64(s: FksSorted, queries, vals_out, found_out, missing: int = 0xFFFFFFFF, stream=None):
    import torch
    _fits(queries.numel(), vals_out=vals_out, found_out=found_out)
    rc = _load().fks_sorted_lookup_u64(s.handle, _dev(queries, _u64_types(), "queries"), queries.numel(),
                                       _dev(vals_out, _u32_types(), "vals_out"),
                                       _dev(found_out, (torch.uint8, torch.bool), "found_out"),
                                       missing & 0xFFFFFFFF, _stream(stream))
    _check(rc, "fks_sorted_lookup_u64")


def fks_sorted_export(s: FksSorted):
    """(keys uint64[n], values uint32[n]) in layout order, as numpy arrays."""
    import numpy as np
    n = s.info()["n"]
    k = np.empty(n, dtype=np.uint64)
    v = np.empty(n, dtype=np.uint32)
    _check(_load().fks_sorted_export(s.handle, k.ctypes.data if n else None, v.ctypes.data if n else None),
           "fks_sorted_export")
    return k, v
