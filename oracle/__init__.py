"""CPU oracle for the static two-level (FKS) hash map -- test infrastructure.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does, and the oracle never
imports the product library.

Modules:
  ``fks_oracle.c`` -- plain sequential C implementation of the construction of
                      Section 2.2-2.3 (make_1 / make_2) and the membership test
                      of Section 2.2, loaded here through ctypes.
  ``spec``         -- the same fixed readings in pure Python integers, for
                      tiny inputs and for pinning the primitives.
  ``search_oracle.c`` -- the comparison maps of Section 4: a sorted array with
                      binary search, and the Eytzinger (level-order) tree of
                      the same keys, built by the recursive in-order walk.
  ``rounds``       -- the sortless flattened construction of Section 2.5 in
                      numpy, written from the paper's data-parallel vocabulary
                      (Figure 1), to show it picks the same level-two
                      constants as the per-bucket make_2.
  ``values``       -- mapping a function over a map's values and reducing them
                      (Section 1), by their plain definitions over the pairs.
"""
from .cbind import (OracleMap, build_u64, build_u64_v64, build_u64_dedup, build_bytes, liboracle, ensure_built,
                    splitmix, hash32, fingerprint, level1_consts, level2_consts,
                    batch_seed, search_build, search_lookup, OK, EINVAL, ENOMEM, EDUPKEY, EBUILD,
                    OracleError)

__all__ = ["OracleMap", "build_u64", "build_u64_v64", "build_u64_dedup", "build_bytes", "liboracle", "ensure_built",
           "splitmix", "hash32", "fingerprint", "level1_consts", "level2_consts",
           "batch_seed", "search_build", "search_lookup", "OK", "EINVAL", "ENOMEM", "EDUPKEY", "EBUILD", "OracleError"]
