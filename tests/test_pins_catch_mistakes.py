"""The pins are strong enough: plausible mistakes planted in (copies of) the oracle's
primitives and tables are caught.  Everything here runs on the CPU; nothing is
planted in the product library."""
import numpy as np
import pytest

import oracle
from oracle import spec
from paper_2508_11443_amd import workloads
from tests import fkscheck
from tests import test_oracle_primitives as P

M64 = (1 << 64) - 1


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


HASH_MUTANTS = {
    "a0/a1 swapped": lambda a0, a1, b, x: spec.hash32(a1, a0, b, x),
    "additive constant dropped": lambda a0, a1, b, x: spec.hash32(a0, a1, 0, x),
    "shift by 31": lambda a0, a1, b, x: (((a0 * (x & 0xFFFFFFFF) + a1 * (x >> 32) + b) & M64) >> 31) & 0xFFFFFFFF,
    "high word ignored": lambda a0, a1, b, x: spec.hash32(a0, 0, b, x & 0xFFFFFFFF),
    "low 32 bits kept": lambda a0, a1, b, x: (a0 * (x & 0xFFFFFFFF) + a1 * (x >> 32) + b) & 0xFFFFFFFF,
}


@pytest.mark.parametrize("name", sorted(HASH_MUTANTS))
def test_hash_mutants_fail_pins(name):
    assert _fails(P.pin_hash_special_cases, HASH_MUTANTS[name])


SPLITMIX_MUTANTS = {
    "counter off by one": lambda s, i: spec.fin(s + i * spec.GAMMA),
    "wrong first shift": lambda s, i: (lambda z: (lambda z: (lambda z: z ^ (z >> 31))(((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64))(((z ^ (z >> 29)) * 0xBF58476D1CE4E5B9) & M64))((s + (i + 1) * spec.GAMMA) & M64),
    "last xorshift dropped": lambda s, i: (lambda z: ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64)(((((s + (i + 1) * spec.GAMMA) & M64) ^ (((s + (i + 1) * spec.GAMMA) & M64) >> 30)) * 0xBF58476D1CE4E5B9) & M64),
}


@pytest.mark.parametrize("name", sorted(SPLITMIX_MUTANTS))
def test_splitmix_mutants_fail_pins(name):
    assert _fails(P.pin_splitmix_vector, SPLITMIX_MUTANTS[name])


FP_MUTANTS = {
    "no length seed": lambda d, b: (lambda acc: acc)(
        __import__("functools").reduce(lambda a, w: (a * b + w) % spec.P61, spec.words32(d), 0)),
    "big-endian words": lambda d, b: __import__("functools").reduce(
        lambda a, w: (a * b + w) % spec.P61,
        [int.from_bytes((d[k:k + 4] + b"\0\0\0")[:4], "big") for k in range(0, len(d), 4)], len(d) % spec.P61),
    "modulus 2^61": lambda d, b: __import__("functools").reduce(
        lambda a, w: (a * b + w) % (1 << 61), spec.words32(d), len(d)),
}


@pytest.mark.parametrize("name", sorted(FP_MUTANTS))
def test_fingerprint_mutants_fail_pins(name):
    assert _fails(P.pin_fingerprint, FP_MUTANTS[name])


def _table(n=3000, sigma=4):
    keys = workloads.unique_u64(n, 12, 0.5)
    vals = np.arange(n, dtype=np.uint32)
    m = oracle.build_u64(keys, vals, sigma)
    h, s = m.export()
    return keys, vals, sigma, m.r, h.copy(), s.copy()


def test_clean_table_passes():
    keys, vals, sigma, r, h, s = _table()
    fkscheck.check_table(keys, vals, sigma, r, h, s)


def _mut_inclusive_base(h, s, n):
    hh = h.reshape(-1, 16).copy()
    base = hh[:, 0:4].copy().view(np.uint32).ravel()
    sizes = hh[:, 4:8].copy().view(np.uint32).ravel()
    first = (sizes & 15).astype(np.uint32)
    base = base + first * first
    hh[:, 0:4] = base.view(np.uint8).reshape(-1, 4)
    return hh.ravel(), s


def _mut_t_plus_one(h, s, n):
    hh = h.reshape(-1, 16).copy()
    base, sizes, t = fkscheck.decode_header(h, n)
    j = int(np.nonzero(sizes[:n] >= 2)[0][0])
    hh[j // 8, 8 + j % 8] += 1
    return hh.ravel(), s


def _mut_t_not_minimal(h, s, n):
    # pretend the first bucket whose minimal trial is 0 had needed trial 1 (re-place it)
    keys, vals, sigma, r, _, _ = _table()
    base, sizes, t = fkscheck.decode_header(h, n)
    hh = h.reshape(-1, 16).copy()
    a0, a1, b, _ = spec.level1_consts(sigma, r)
    C1 = spec.level2_consts(sigma, r, 1)
    g = np.array([spec.hash32(a0, a1, b, int(k)) % n for k in keys])
    offs = np.concatenate([[0], np.cumsum(sizes[:n] ** 2)])
    cells = s.reshape(-1, 16).copy()
    for j in np.nonzero((sizes[:n] >= 2) & (t[:n] == 0))[0]:
        members = np.nonzero(g == j)[0]
        pos = [offs[j] + spec.hash32(*C1, int(keys[i])) % (sizes[j] ** 2) for i in members]
        if len(set(pos)) == len(pos):
            hh[j // 8, 8 + j % 8] = 1
            lo, hi = offs[j], offs[j + 1]
            new = np.zeros((hi - lo, 16), np.uint8)
            filled = np.zeros(hi - lo, bool)
            for i, p in zip(members, pos):
                new[p - lo, 0:8] = np.array([keys[i]], np.uint64).view(np.uint8)
                new[p - lo, 8:12] = np.array([vals[i]], np.uint32).view(np.uint8)
                filled[p - lo] = True
            first = int(np.nonzero(filled)[0][0])
            new[~filled] = new[first]
            cells[lo:hi] = new
            return hh.ravel(), cells.ravel()
    raise RuntimeError("no candidate bucket")


def _mut_fill_highest(h, s, n):
    base, sizes, t = fkscheck.decode_header(h, n)
    cells = s.reshape(-1, 16).copy()
    offs = np.concatenate([[0], np.cumsum(sizes[:n] ** 2)])
    for j in np.nonzero(sizes[:n] >= 2)[0]:
        lo, hi = offs[j], offs[j + 1]
        blk = cells[lo:hi]
        uniq = np.unique(blk, axis=0)
        if uniq.shape[0] >= 2 and hi - lo > uniq.shape[0]:
            # rows equal to the lowest occupied cell but not the lowest itself are fills
            first = blk[0] if True else None
            occupied_last = None
            for p in range(hi - lo - 1, -1, -1):
                if p == 0 or not (blk[p] == blk[0]).all():
                    occupied_last = p
                    break
            fills = [p for p in range(1, hi - lo) if (blk[p] == blk[0]).all()]
            if fills and occupied_last:
                for p in fills:
                    blk[p] = blk[occupied_last]
                cells[lo:hi] = blk
                return h, cells.ravel()
    raise RuntimeError("no candidate bucket")


def _mut_swap_values(h, s, n):
    cells = s.reshape(-1, 16).copy()
    ck = cells[:, 0:8].copy().view(np.uint64).ravel()
    a, b = 0, int(np.nonzero(ck != ck[0])[0][0])
    va, vb = cells[a, 8:12].copy(), cells[b, 8:12].copy()
    cells[a, 8:12], cells[b, 8:12] = vb, va
    return h, cells.ravel()


def _mut_sizes_shifted(h, s, n):
    hh = h.reshape(-1, 16).copy()
    sizes = hh[:, 4:8].copy().view(np.uint32).ravel()
    sizes = np.roll(sizes, 1)
    hh[:, 4:8] = sizes.view(np.uint8).reshape(-1, 4)
    return hh.ravel(), s


def _mut_tags_zero(h, s, n):
    # a one-key bucket's byte left at its trial (0) instead of its key's tag
    hh = h.reshape(-1, 16).copy()
    _, sizes, _ = fkscheck.decode_header(h, n)
    one = np.nonzero(sizes[:n] == 1)[0]
    hh[one // 8, 8 + one % 8] = 0
    return hh.ravel(), s


def _mut_tag_of_trial_one(h, s, n):
    # the tag taken from trial 1's hash instead of trial 0's
    keys, vals, sigma, r, _, _ = _table()
    hh = h.reshape(-1, 16).copy()
    _, sizes, _ = fkscheck.decode_header(h, n)
    a0, a1, b, _ = spec.level1_consts(sigma, r)
    C1 = spec.level2_consts(sigma, r, 1)
    for k in keys:
        j = spec.hash32(a0, a1, b, int(k)) % n
        if sizes[j] == 1:
            hh[j // 8, 8 + j % 8] = spec.hash32(*C1, int(k)) >> 24
    return hh.ravel(), s


def _mut_tag_low_bits(h, s, n):
    # the low 8 bits of the trial-0 hash instead of the top 8
    keys, vals, sigma, r, _, _ = _table()
    hh = h.reshape(-1, 16).copy()
    _, sizes, _ = fkscheck.decode_header(h, n)
    a0, a1, b, _ = spec.level1_consts(sigma, r)
    C0 = spec.level2_consts(sigma, r, 0)
    for k in keys:
        j = spec.hash32(a0, a1, b, int(k)) % n
        if sizes[j] == 1:
            hh[j // 8, 8 + j % 8] = spec.hash32(*C0, int(k)) & 0xFF
    return hh.ravel(), s


TABLE_MUTANTS = {
    "one-key bucket without its tag": _mut_tags_zero,
    "tag from trial 1": _mut_tag_of_trial_one,
    "tag from the low bits": _mut_tag_low_bits,
    "inclusive presum for bases": _mut_inclusive_base,
    "trial index off by one": _mut_t_plus_one,
    "non-minimal trial": _mut_t_not_minimal,
    "fill with highest occupied cell": _mut_fill_highest,
    "values of two cells swapped": _mut_swap_values,
    "sizes of a wrong group": _mut_sizes_shifted,
}


@pytest.mark.parametrize("name", sorted(TABLE_MUTANTS))
def test_table_mutants_fail_checks(name):
    keys, vals, sigma, r, h, s = _table()
    h2, s2 = TABLE_MUTANTS[name](h, s, keys.size)
    assert _fails(fkscheck.check_table, keys, vals, sigma, r, h2, s2)


# ---- map and reduce over values ------------------------------------------------------

from oracle import values as OV  # noqa: E402
from tests import test_oracle_values as PV  # noqa: E402


def _map_64_always(v, op, a, b, table, width):
    return OV.map_values(v, op, a, b, table, 64)


def _map_affine_swapped(v, op, a, b, table, width):
    return OV.map_values(v, op, b, a, table, width) if op == OV.VOP_AFFINE else OV.map_values(v, op, a, b, table, width)


def _map_affine_no_b(v, op, a, b, table, width):
    return OV.map_values(v, OV.VOP_MUL, a, 0, table, width) if op == OV.VOP_AFFINE else \
        OV.map_values(v, op, a, b, table, width)


def _map_gather_wraps(v, op, a, b, table, width):
    if op == OV.VOP_GATHER:
        t = np.asarray(table)
        return t[np.asarray(v).astype(np.int64) % t.size]
    return OV.map_values(v, op, a, b, table, width)


MAP_MUTANTS = {
    "32-bit values kept to 64 bits": _map_64_always,
    "affine operands swapped": _map_affine_swapped,
    "affine additive term dropped": _map_affine_no_b,
    "gather index wrapped instead of refused": _map_gather_wraps,
}


@pytest.mark.parametrize("name", sorted(MAP_MUTANTS))
def test_map_values_mutants_fail_pins(name):
    assert _fails(PV.pin_map_values, MAP_MUTANTS[name])


REDUCE_MUTANTS = {
    "min of an empty map is 0": lambda v, op, w: 0 if (op == OV.VRED_MIN and np.asarray(v).size == 0)
    else OV.reduce_values(v, op, w),
    "xor folded as or": lambda v, op, w: int(np.bitwise_or.reduce(np.asarray(v).astype(np.uint64)))
    if (op == OV.VRED_XOR and np.asarray(v).size) else OV.reduce_values(v, op, w),
    "last value dropped": lambda v, op, w: OV.reduce_values(np.asarray(v)[:-1], op, w),
    "max folded as min": lambda v, op, w: OV.reduce_values(v, OV.VRED_MIN if op == OV.VRED_MAX else op, w),
}


@pytest.mark.parametrize("name", sorted(REDUCE_MUTANTS))
def test_reduce_values_mutants_fail_pins(name):
    assert _fails(PV.pin_reduce_values, REDUCE_MUTANTS[name])
