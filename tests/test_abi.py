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
    assert lib.fks_build_u64(None, None, 5, 1, None, None, ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_build_u64(None, None, 1 << 30, 1, None, None, ctypes.byref(out)) == fks.FKS_EINVAL
    bad = fks.fks_params(4, 0, 16, 0)
    assert lib.fks_build_u64(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 1, ctypes.byref(bad), None,
                             ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_lookup_u64(None, None, 0, None, None, 0, None) == fks.FKS_EINVAL
    assert lib.fks_info(None, None) == fks.FKS_EINVAL
    assert lib.fks_map_values(None, fks.FKS_VOP_ADD, 1, 0, None, 0, None, ctypes.byref(out)) == fks.FKS_EINVAL
    assert lib.fks_reduce_values(None, fks.FKS_VRED_SUM, None, None) == fks.FKS_EINVAL
    assert lib.fks_probe_random_reads(1 << 20, 0, 16, None, None) == fks.FKS_EINVAL
    assert out.value is None   # out-parameters untouched on failure
    lib.fks_destroy(None)
