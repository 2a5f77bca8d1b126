"""ctypes binding of the C oracles (``fks_oracle.c``, ``search_oracle.c``).  Test
infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fks_oracle.c"), os.path.join(_HERE, "search_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
# the same sources with their independent loops run by OpenMP on every host core
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, EINVAL, ENOMEM, EDUPKEY, EBUILD = 0, -1, -2, -3, -4
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDUPKEY: "EDUPKEY", EBUILD: "EBUILD"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle build failed: {_NAMES.get(code, code)}")
        self.code = code


def compile_oracle() -> str:
    """Compile the C oracles into ``oracle/liboracle.so`` (gcc, plain -O2, sequential) and
    ``oracle/liboracle_omp.so`` (the same sources with -fopenmp)."""
    for lib, extra in ((_LIB, ["-Wno-unknown-pragmas"]), (_LIB_OMP, ["-fopenmp"])):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", *extra, "-shared", "-fPIC",
                               "-o", tmp] + _SRCS)
        os.replace(tmp, lib)
    return _LIB


def ensure_built() -> str:
    newest = max(os.path.getmtime(f) for f in _SRCS)
    if any(not os.path.exists(p) or os.path.getmtime(p) < newest for p in (_LIB, _LIB_OMP)):
        compile_oracle()
    return _LIB


_lib = None
_lib_omp = None


def liboracle_omp():
    """The OpenMP build: the same functions, their independent loops on every host core
    (OMP_NUM_THREADS threads); its results are those of the sequential build."""
    global _lib_omp
    if _lib_omp is None:
        ensure_built()
        _lib_omp = _configure(ctypes.CDLL(_LIB_OMP))
    return _lib_omp


def threads(omp: bool) -> int:
    """Host threads the oracle's loops run on."""
    return int((liboracle_omp() if omp else liboracle()).oracle_threads())


def liboracle():
    global _lib
    if _lib is None:
        _lib = _configure(ctypes.CDLL(ensure_built()))
    return _lib


def _configure(lib):
    """Argument and result types of every exported function."""
    u64, u32, vp, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    lib.oracle_splitmix.restype = u64
    lib.oracle_splitmix.argtypes = [u64, u64]
    lib.oracle_hash.restype = u32
    lib.oracle_hash.argtypes = [u64, u64, u64, u64]
    lib.oracle_level1_consts.restype = None
    lib.oracle_level1_consts.argtypes = [u64, u32, vp]
    lib.oracle_level2_consts.restype = None
    lib.oracle_level2_consts.argtypes = [u64, u32, u32, vp]
    lib.oracle_fingerprint.restype = u64
    lib.oracle_fingerprint.argtypes = [vp, u64, u64]
    lib.oracle_build_u64.restype = i32
    lib.oracle_build_u64.argtypes = [vp, vp, u64, u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.oracle_build_u64_dedup.restype = i32
    lib.oracle_build_u64_dedup.argtypes = [vp, vp, u64, u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.oracle_build_bytes.restype = i32
    lib.oracle_build_bytes.argtypes = [vp, vp, vp, u64, u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.oracle_lookup_u64.restype = i32
    lib.oracle_lookup_u64.argtypes = [vp, vp, u64, vp, vp, u32]
    lib.oracle_lookup_bytes.restype = i32
    lib.oracle_lookup_bytes.argtypes = [vp, vp, vp, u64, vp, vp, u32]
    lib.oracle_info.restype = None
    lib.oracle_info.argtypes = [vp, vp]
    lib.oracle_export.restype = None
    lib.oracle_export.argtypes = [vp, vp, vp]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [vp]
    lib.oracle_batch_seed.restype = u64
    lib.oracle_batch_seed.argtypes = [u64, u64]
    lib.oracle_build_u64_v64.restype = i32
    lib.oracle_build_u64_v64.argtypes = [vp, vp, u64, u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.oracle_lookup_u64_v64.restype = i32
    lib.oracle_lookup_u64_v64.argtypes = [vp, vp, u64, vp, vp, u64]
    lib.oracle_search_build.restype = i32
    lib.oracle_search_build.argtypes = [vp, vp, u64, u32, vp, vp]
    lib.oracle_search_lookup.restype = i32
    lib.oracle_search_lookup.argtypes = [vp, vp, u64, u32, vp, u64, vp, vp, u32]
    lib.oracle_threads.restype = i32
    lib.oracle_threads.argtypes = []
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def splitmix(sigma: int, i: int) -> int:
    return int(liboracle().oracle_splitmix(sigma, i))


def hash32(a0: int, a1: int, b: int, x: int) -> int:
    return int(liboracle().oracle_hash(a0, a1, b, x))


def level1_consts(sigma: int, r: int):
    out = np.zeros(4, np.uint64)
    liboracle().oracle_level1_consts(sigma, r, _ptr(out))
    return tuple(int(v) for v in out)


def level2_consts(sigma: int, r: int, t: int):
    out = np.zeros(3, np.uint64)
    liboracle().oracle_level2_consts(sigma, r, t, _ptr(out))
    return tuple(int(v) for v in out)


def fingerprint(data: bytes, beta: int) -> int:
    buf = np.frombuffer(data, np.uint8) if data else np.zeros(1, np.uint8)
    return int(liboracle().oracle_fingerprint(_ptr(buf), len(data), beta))


def batch_seed(batch_sigma: int, m: int) -> int:
    return int(liboracle().oracle_batch_seed(batch_sigma, m))


INFO_FIELDS = ("n", "S", "r", "T", "c", "kind", "beta", "a0", "a1", "a2",
               "rejected_size", "rejected_space", "rejected_exhausted", "level2_trials")


class OracleMap:
    """A map built by the C oracle; owns the C object."""

    def __init__(self, handle: int, lib=None):
        self._lib = lib if lib is not None else liboracle()
        self._h = ctypes.c_void_p(handle)
        info = np.zeros(len(INFO_FIELDS), np.uint64)
        self._lib.oracle_info(self._h, _ptr(info))
        self.info = {k: int(v) for k, v in zip(INFO_FIELDS, info)}
        self.n, self.S, self.r = self.info["n"], self.info["S"], self.info["r"]
        self.kind = {0: "u64", 1: "bytes", 2: "u64v64"}[self.info["kind"]]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.oracle_free(h)
            self._h = None

    def export(self):
        """(header u8[16*ceil(n/8)], slots u8[16*S]) exactly as the oracle laid them out."""
        ng = (self.n + 7) // 8
        header = np.zeros(16 * ng, np.uint8)
        slots = np.zeros(16 * self.S, np.uint8)
        self._lib.oracle_export(self._h, _ptr(header), _ptr(slots))
        return header, slots

    def lookup(self, queries: np.ndarray, missing: int = 0xFFFFFFFF):
        q = np.ascontiguousarray(queries, np.uint64)
        vals = np.zeros(q.size, np.uint32)
        found = np.zeros(q.size, np.uint8)
        rc = self._lib.oracle_lookup_u64(self._h, _ptr(q), q.size, _ptr(vals), _ptr(found), missing)
        if rc:
            raise OracleError(rc)
        return vals, found

    def lookup_v64(self, queries: np.ndarray, missing: int = 2**64 - 1):
        q = np.ascontiguousarray(queries, np.uint64)
        vals = np.zeros(q.size, np.uint64)
        found = np.zeros(q.size, np.uint8)
        rc = self._lib.oracle_lookup_u64_v64(self._h, _ptr(q), q.size, _ptr(vals), _ptr(found), missing)
        if rc:
            raise OracleError(rc)
        return vals, found

    def lookup_bytes(self, offsets: np.ndarray, data: np.ndarray, missing: int = 0xFFFFFFFF):
        off = np.ascontiguousarray(offsets, np.int64)
        buf = np.ascontiguousarray(data, np.uint8)
        if buf.size == 0:
            buf = np.zeros(1, np.uint8)
        m = off.size - 1
        vals = np.zeros(m, np.uint32)
        found = np.zeros(m, np.uint8)
        rc = self._lib.oracle_lookup_bytes(self._h, _ptr(off), _ptr(buf), m, _ptr(vals),
                                             _ptr(found), missing)
        if rc:
            raise OracleError(rc)
        return vals, found


def build_u64(keys: np.ndarray, vals: np.ndarray, sigma: int, c: int = 4, T: int = 64,
              R: int = 16, omp: bool = False) -> OracleMap:
    """With omp, the OpenMP build of the oracle builds (and later queries) the map."""
    k = np.ascontiguousarray(keys, np.uint64)
    v = np.ascontiguousarray(vals, np.uint32)
    assert k.size == v.size
    lib = liboracle_omp() if omp else liboracle()
    h = ctypes.c_void_p()
    rc = lib.oracle_build_u64(_ptr(k), _ptr(v), k.size, sigma, c, T, R, ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    return OracleMap(h.value, lib)


def build_u64_v64(keys: np.ndarray, vals: np.ndarray, sigma: int, c: int = 4, T: int = 64,
                  R: int = 16) -> OracleMap:
    """64-bit values: the value's high half sits in the cell's aux word."""
    k = np.ascontiguousarray(keys, np.uint64)
    v = np.ascontiguousarray(vals, np.uint64)
    assert k.size == v.size
    h = ctypes.c_void_p()
    rc = liboracle().oracle_build_u64_v64(_ptr(k), _ptr(v), k.size, sigma, c, T, R, ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    return OracleMap(h.value)


def build_u64_dedup(keys: np.ndarray, vals: np.ndarray, sigma: int, c: int = 4, T: int = 64,
                    R: int = 16) -> OracleMap:
    """from_array: repeated keys keep the value of their first occurrence."""
    k = np.ascontiguousarray(keys, np.uint64)
    v = np.ascontiguousarray(vals, np.uint32)
    assert k.size == v.size
    h = ctypes.c_void_p()
    rc = liboracle().oracle_build_u64_dedup(_ptr(k), _ptr(v), k.size, sigma, c, T, R, ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    return OracleMap(h.value)


def build_bytes(offsets: np.ndarray, data: np.ndarray, vals: np.ndarray, sigma: int, c: int = 4,
                T: int = 64, R: int = 16, omp: bool = False) -> OracleMap:
    off = np.ascontiguousarray(offsets, np.int64)
    buf = np.ascontiguousarray(data, np.uint8)
    if buf.size == 0:
        buf = np.zeros(1, np.uint8)
    v = np.ascontiguousarray(vals, np.uint32)
    n = off.size - 1
    assert v.size == n
    lib = liboracle_omp() if omp else liboracle()
    h = ctypes.c_void_p()
    rc = lib.oracle_build_bytes(_ptr(off), _ptr(buf), _ptr(v), n, sigma, c, T, R, ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    return OracleMap(h.value, lib)


def search_build(keys: np.ndarray, vals: np.ndarray, layout: int):
    """Sorted (layout 0) or Eytzinger (layout 1) arrays of the pairs; raises on
    duplicate keys."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ok = np.empty(keys.size, dtype=np.uint64)
    ov = np.empty(keys.size, dtype=np.uint32)
    rc = liboracle().oracle_search_build(_ptr(keys), _ptr(vals), keys.size, layout, _ptr(ok), _ptr(ov))
    if rc != OK:
        raise OracleError(rc)
    return ok, ov


def search_lookup(lkeys: np.ndarray, lvals: np.ndarray, layout: int, q: np.ndarray, missing: int = 0xFFFFFFFF):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    vals = np.empty(q.size, dtype=np.uint32)
    found = np.empty(q.size, dtype=np.uint8)
    rc = liboracle().oracle_search_lookup(_ptr(lkeys), _ptr(lvals), lkeys.size, layout, _ptr(q), q.size,
                                          _ptr(vals), _ptr(found), missing)
    if rc != OK:
        raise OracleError(rc)
    return vals, found.astype(bool)
