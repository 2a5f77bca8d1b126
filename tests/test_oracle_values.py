"""Pins of the oracle's map and reduce over values (Section 1's operations on a map's values).

Each check is fixed by arithmetic, not by the oracle's own formula: closed forms of sums and
xors over 0..n-1, inverse operations that must give the identity in the value width (a wrong
width or a swapped operand fails them), the identities of the folds, and the map-then-reduce
law sum(v + a) = sum(v) + n*a."""
import numpy as np
import pytest

from oracle import values as ov


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 1000, 1 << 16, (1 << 16) + 3])
def test_sum_and_xor_of_0_to_n_minus_1(n):
    v = np.random.default_rng(n).permutation(np.arange(n, dtype=np.uint64))
    assert ov.reduce_values(v, ov.VRED_SUM) == n * (n - 1) // 2
    # xor of 0..m is m, 1, m+1, 0 for m = 0, 1, 2, 3 mod 4
    m = n - 1
    expect = 0 if n == 0 else [m, 1, m + 1, 0][m % 4]
    assert ov.reduce_values(v, ov.VRED_XOR) == expect


@pytest.mark.parametrize("width", [32, 64])
def test_min_max_and_identities(width):
    v = np.random.default_rng(width).permutation(np.arange(10, 1010, dtype=np.uint64))
    assert ov.reduce_values(v, ov.VRED_MIN, width) == 10
    assert ov.reduce_values(v, ov.VRED_MAX, width) == 1009
    empty = np.zeros(0, np.uint64)
    assert ov.reduce_values(empty, ov.VRED_MIN, width) == (1 << width) - 1
    for op in (ov.VRED_SUM, ov.VRED_MAX, ov.VRED_XOR):
        assert ov.reduce_values(empty, op, width) == 0


def test_sum_wraps_modulo_2_64():
    v = np.array([1 << 63, 1 << 63, 5], np.uint64)
    assert ov.reduce_values(v, ov.VRED_SUM, 64) == 5


@pytest.mark.parametrize("width", [32, 64])
def test_add_then_its_inverse_is_the_identity(width):
    rng = np.random.default_rng(3)
    v = rng.integers(0, 1 << width, size=5000, dtype=np.uint64)
    a = int(rng.integers(1, 1 << width, dtype=np.uint64))
    once = ov.map_values(v, ov.VOP_ADD, a, width=width)
    back = ov.map_values(once, ov.VOP_ADD, (1 << width) - a, width=width)
    assert (back.astype(np.uint64) == v).all()
    assert not (once.astype(np.uint64) == v).all()


@pytest.mark.parametrize("width", [32, 64])
def test_mul_by_an_odd_number_then_its_inverse_is_the_identity(width):
    rng = np.random.default_rng(4)
    v = rng.integers(0, 1 << width, size=5000, dtype=np.uint64)
    a = int(rng.integers(0, 1 << (width - 1), dtype=np.uint64)) * 2 + 1
    inv = pow(a, -1, 1 << width)
    back = ov.map_values(ov.map_values(v, ov.VOP_MUL, a, width=width), ov.VOP_MUL, inv, width=width)
    assert (back.astype(np.uint64) == v).all()


@pytest.mark.parametrize("width", [32, 64])
def test_affine_is_mul_then_add(width):
    rng = np.random.default_rng(5)
    v = rng.integers(0, 1 << width, size=2000, dtype=np.uint64)
    a, b = 0x9E3779B97F4A7C15 & ((1 << width) - 1), 12345
    two_steps = ov.map_values(ov.map_values(v, ov.VOP_MUL, a, width=width), ov.VOP_ADD, b, width=width)
    assert (ov.map_values(v, ov.VOP_AFFINE, a, b, width=width) == two_steps).all()
    # b is the additive term: v = 0 maps to b
    assert int(ov.map_values(np.zeros(1, np.uint64), ov.VOP_AFFINE, a, b, width=width)[0]) == b


def test_xor_twice_and_gather_through_a_reversal():
    v = np.arange(100, dtype=np.uint32)
    assert (ov.map_values(ov.map_values(v, ov.VOP_XOR, 0xA5A5A5A5), ov.VOP_XOR, 0xA5A5A5A5) == v).all()
    table = np.arange(100, dtype=np.uint32)[::-1].copy()
    assert (ov.map_values(v, ov.VOP_GATHER, table=table) == 99 - v).all()
    with pytest.raises(ValueError):
        ov.map_values(np.array([100], np.uint32), ov.VOP_GATHER, table=table)


def test_sum_after_add_is_sum_plus_n_times_a():
    v = np.random.default_rng(6).integers(0, 1 << 32, size=777, dtype=np.uint64).astype(np.uint32)
    a = 0xDEADBEEF
    mapped = ov.map_values(v, ov.VOP_ADD, a)
    # each mapped value is (v + a) mod 2^32: the sums differ by n*a minus 2^32 per wrap
    wraps = int(((v.astype(np.uint64) + a) >> 32).sum())
    assert ov.reduce_values(mapped, ov.VRED_SUM) == ov.reduce_values(v, ov.VRED_SUM) + 777 * a - (wraps << 32)
