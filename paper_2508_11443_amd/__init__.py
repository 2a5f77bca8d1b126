"""Static two-level (FKS) hash maps built and queried on AMD Instinct MI355X (gfx950).

The product is the C-ABI library ``libfks.so`` (declared in include/fks.h, HIP
kernels under ``csrc/``); ``fks`` is its thin Python binding and ``workloads``
holds the seeded synthetic inputs.
"""
__all__ = ["fks", "workloads", "build_lib"]
