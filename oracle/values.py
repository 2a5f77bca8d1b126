"""Map and reduce over the values of a map, by their plain definitions.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product.

Section 1 motivates hash maps in an array language by the operations they share
with arrays: mapping a function over the values, and reducing the values to a
single value.  A map is a finite function from its keys to values, so:

  * mapping f over a map with pairs (k, v) gives the map with pairs (k, f(v)) --
    its table is therefore the table that the construction of Section 2.2 (the
    C oracle's build) writes for those pairs; ``map_values`` computes the new
    value array;
  * reducing a map with an associative, commutative operation folds the
    operation over the values of its keys, each key counted once;
    ``reduce_values`` folds over the input value array.

Arithmetic is modular in the value width w (32 bits for maps with uint32
values, 64 for maps with uint64 values).  The operation codes are those of the
library's C interface.
"""
from __future__ import annotations

import numpy as np

VOP_ADD, VOP_MUL, VOP_XOR, VOP_AFFINE, VOP_GATHER = 0, 1, 2, 3, 4
VRED_SUM, VRED_MIN, VRED_MAX, VRED_XOR = 0, 1, 2, 3


def _mask(width: int) -> int:
    assert width in (32, 64)
    return (1 << width) - 1


def map_values(vals: np.ndarray, op: int, a: int = 0, b: int = 0, table=None, width: int = 32) -> np.ndarray:
    """f(v) for every value v, modulo 2^width (uint32 or uint64 array, like the input).
    VOP_GATHER reads table[v]; a value outside the table raises ValueError."""
    m = _mask(width)
    out_t = np.uint32 if width == 32 else np.uint64
    v = np.asarray(vals).astype(np.uint64)
    a64, b64 = np.uint64(a & m), np.uint64(b & m)
    # numpy's uint64 arithmetic wraps modulo 2^64; reducing modulo 2^32 afterwards
    # gives the 32-bit modular result
    with np.errstate(over="ignore"):
        if op == VOP_ADD:
            r = v + a64
        elif op == VOP_MUL:
            r = v * a64
        elif op == VOP_XOR:
            r = v ^ a64
        elif op == VOP_AFFINE:
            r = v * a64 + b64
        elif op == VOP_GATHER:
            t = np.asarray(table if table is not None else np.zeros(0, out_t)).astype(np.uint64)
            if v.size and int(v.max()) >= t.size:
                raise ValueError("a value lies outside the gather table")
            r = t[v.astype(np.int64)] if v.size else v
        else:
            raise ValueError(f"unknown value operation {op}")
    return (r & np.uint64(m)).astype(out_t)


def identity(op: int, width: int = 32) -> int:
    """The fold's result on a map without keys."""
    return _mask(width) if op == VRED_MIN else 0


def reduce_values(vals: np.ndarray, op: int, width: int = 32) -> int:
    """Fold of op over the values (SUM modulo 2^64, MIN, MAX, XOR)."""
    v = np.asarray(vals).astype(np.uint64)
    if v.size == 0:
        return identity(op, width)
    if op == VRED_SUM:
        with np.errstate(over="ignore"):
            return int(np.add.reduce(v, dtype=np.uint64))
    if op == VRED_MIN:
        return int(v.min())
    if op == VRED_MAX:
        return int(v.max())
    if op == VRED_XOR:
        return int(np.bitwise_xor.reduce(v))
    raise ValueError(f"unknown reduction {op}")
