"""The C ABI library loads on the CPU host and exports every entry point that
include/fks.h declares; the Python binding names the same functions.  No compute
calls: nothing here needs a GPU."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(fks_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def declared_arities():
    """{function name: number of parameters} of every declaration in the headers."""
    out = {}
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(fks_\w+)\s*\(([^)]*)\)\s*;", text, flags=re.M):
            params = [p.strip() for p in m.group(2).split(",") if p.strip()]
            out[m.group(1)] = 0 if params == ["void"] else len(params)
    return out


@pytest.fixture(scope="module")
def lib():
    from paper_2508_11443_amd import fks
    if not os.path.exists(fks.LIB_PATH):
        from paper_2508_11443_amd import build_lib
        build_lib.build()
    return fks.library()


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("fks_build_u64", "fks_build_bytes", "fks_lookup_u64", "fks_contains_u64",
                 "fks_lookup_bytes", "fks_contains_bytes", "fks_export", "fks_destroy", "fks_info"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2508_11443_amd import fks
    out = subprocess.run(["nm", "-D", "--defined-only", fks.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared_functions() - exported
    assert not missing, missing
    for name in declared_functions():
        assert hasattr(lib, name)


def test_binding_covers_the_header(lib):
    from paper_2508_11443_amd import fks
    bound = {name for name, _, _ in fks.SIGNATURES}
    assert declared_functions() <= bound | {n for n in declared_functions() if n.startswith("fks_server")}, \
        declared_functions() - bound


def test_binding_arities_match_the_header():
    """Every ctypes signature passes as many arguments as the C declaration takes."""
    from paper_2508_11443_amd import fks
    arity = declared_arities()
    for name, _, args in fks.SIGNATURES:
        assert arity[name] == len(args), (name, arity[name], len(args))


def test_host_only_entry_points(lib):
    import ctypes
    from paper_2508_11443_amd import fks
    p = fks.fks_params()
    lib.fks_params_default(ctypes.byref(p))
    assert (p.c, p.T, p.R, p.schedule) == (4, 64, 16, 0)
    assert lib.fks_strerror(0) == b"ok"
    assert lib.fks_strerror(fks.FKS_EDUPKEY).startswith(b"duplicate")
    assert lib.fks_version() >= 10000
    # argument checks that return before any device work
    out = ctypes.c_void_p()
    assert lib.fks_build_u64(None, None, 5, 1, None, None, None, ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_build_u64(None, None, 1 << 30, 1, None, None, None, ctypes.byref(out)) == fks.FKS_EINVAL
    bad = fks.fks_params(4, 0, 16, 0)
    assert lib.fks_build_u64(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 1, ctypes.byref(bad), None, None,
                             ctypes.byref(out)) == fks.FKS_EINVAL
    # an allocator must set both of its functions
    half = fks.fks_allocator()
    half.alloc = fks.ALLOC_FN(lambda nbytes, stream, user: None)
    for call in (lambda a: lib.fks_build_u64(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 1, None, a, None,
                                             ctypes.byref(out)),
                 lambda a: lib.fks_build_bytes(ctypes.c_void_p(16), ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 1,
                                               1, None, a, None, ctypes.byref(out)),
                 lambda a: lib.fks_build_u64_v64(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 1, None, a, None,
                                                 ctypes.byref(out)),
                 lambda a: lib.fks_build_u64_from_array(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 1, None, a,
                                                        None, ctypes.byref(out)),
                 lambda a: lib.fks_sorted_build_u64(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 0, a, None,
                                                    ctypes.byref(out))):
        assert call(ctypes.byref(fks.fks_allocator())) == fks.FKS_EINVAL
        assert call(ctypes.byref(half)) == fks.FKS_EINVAL
    offs = (ctypes.c_uint64 * 2)(0, 5)
    assert lib.fks_build_batch_u64(ctypes.c_void_p(16), ctypes.c_void_p(16), offs, 1, 1, None, 0,
                                   ctypes.byref(half), None, ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_lookup_u64(None, None, 0, None, None, 0, None) == fks.FKS_EINVAL
    assert lib.fks_info(None, None) == fks.FKS_EINVAL
    assert lib.fks_map_values(None, fks.FKS_VOP_ADD, 1, 0, None, 0, None, None,
                              ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_reduce_values(None, fks.FKS_VRED_SUM, None, None) == fks.FKS_EINVAL
    assert lib.fks_probe_random_reads(1 << 20, 0, 16, None, None) == fks.FKS_EINVAL
    assert out.value is None   # out-parameters untouched on failure
    lib.fks_destroy(None)
