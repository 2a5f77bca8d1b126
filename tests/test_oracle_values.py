"""Pins of the oracle's map and reduce over values (Section 1's operations on a map's values).

Each check is fixed by arithmetic, not by the oracle's own formula: closed forms of sums and
xors over 0..n-1, inverse operations that must give the identity in the value width (a wrong
width or a swapped operand fails them), the identities of the folds, and the map-then-reduce
law sum(v + a) = sum(v) + n*a less 2^32 per wrapped value.  The pins take the implementation as
an argument so that planted mistakes can be shown to fail them."""
import numpy as np

from oracle import values as ov

SIZES = [0, 1, 2, 3, 4, 5, 1000, 1 << 16, (1 << 16) + 3]


def pin_reduce_values(reduce_values):
    for n in SIZES:
        v = np.random.default_rng(n).permutation(np.arange(n, dtype=np.uint64))
        assert reduce_values(v, ov.VRED_SUM, 32) == n * (n - 1) // 2
        # xor of 0..m is m, 1, m+1, 0 for m = 0, 1, 2, 3 mod 4
        m = n - 1
        assert reduce_values(v, ov.VRED_XOR, 32) == (0 if n == 0 else [m, 1, m + 1, 0][m % 4])
    for width in (32, 64):
        v = np.random.default_rng(width).permutation(np.arange(10, 1010, dtype=np.uint64))
        assert reduce_values(v, ov.VRED_MIN, width) == 10
        assert reduce_values(v, ov.VRED_MAX, width) == 1009
        empty = np.zeros(0, np.uint64)
        assert reduce_values(empty, ov.VRED_MIN, width) == (1 << width) - 1
        for op in (ov.VRED_SUM, ov.VRED_MAX, ov.VRED_XOR):
            assert reduce_values(empty, op, width) == 0
    assert reduce_values(np.array([1 << 63, 1 << 63, 5], np.uint64), ov.VRED_SUM, 64) == 5


def pin_map_values(map_values):
    for width in (32, 64):
        rng = np.random.default_rng(width)
        mask = (1 << width) - 1
        v = rng.integers(0, 1 << width, size=5000, dtype=np.uint64)
        # add, then the additive inverse
        a = int(rng.integers(1, 1 << width, dtype=np.uint64))
        once = map_values(v, ov.VOP_ADD, a, 0, None, width)
        assert not (once.astype(np.uint64) == v).all()
        assert (map_values(once, ov.VOP_ADD, (1 << width) - a, 0, None, width).astype(np.uint64) == v).all()
        # multiply by an odd number, then by its inverse modulo 2^width
        a = int(rng.integers(0, 1 << (width - 1), dtype=np.uint64)) * 2 + 1
        inv = pow(a, -1, 1 << width)
        back = map_values(map_values(v, ov.VOP_MUL, a, 0, None, width), ov.VOP_MUL, inv, 0, None, width)
        assert (back.astype(np.uint64) == v).all()
        # affine is multiply then add, and b is the additive term
        a, b = 0x9E3779B97F4A7C15 & mask, 12345
        two = map_values(map_values(v, ov.VOP_MUL, a, 0, None, width), ov.VOP_ADD, b, 0, None, width)
        assert (map_values(v, ov.VOP_AFFINE, a, b, None, width) == two).all()
        assert int(map_values(np.zeros(1, np.uint64), ov.VOP_AFFINE, a, b, None, width)[0]) == b
        # xor twice is the identity
        x = 0xA5A5A5A5A5A5A5A5 & mask
        assert (map_values(map_values(v, ov.VOP_XOR, x, 0, None, width), ov.VOP_XOR, x, 0, None, width)
                .astype(np.uint64) == v).all()
    # gather through a reversal; an index past the table is an error
    v = np.arange(100, dtype=np.uint32)
    table = np.arange(100, dtype=np.uint32)[::-1].copy()
    assert (map_values(v, ov.VOP_GATHER, 0, 0, table, 32) == 99 - v).all()
    try:
        map_values(np.array([100], np.uint32), ov.VOP_GATHER, 0, 0, table, 32)
        raised = False
    except ValueError:
        raised = True
    assert raised, "a gather index past the table must be refused"
    # map then reduce: sum(v + a mod 2^32) = sum(v) + n*a - 2^32 * (values that wrapped)
    v = np.random.default_rng(6).integers(0, 1 << 32, size=777, dtype=np.uint64).astype(np.uint32)
    a = 0xDEADBEEF
    wraps = int(((v.astype(np.uint64) + a) >> 32).sum())
    mapped = map_values(v, ov.VOP_ADD, a, 0, None, 32)
    assert int(mapped.astype(np.uint64).sum()) == int(v.astype(np.uint64).sum()) + 777 * a - (wraps << 32)


def _oracle_map(v, op, a, b, table, width):
    return ov.map_values(v, op, a, b, table, width)


def test_reduce_values_pins():
    pin_reduce_values(ov.reduce_values)


def test_map_values_pins():
    pin_map_values(_oracle_map)


def test_own_cells_are_exactly_the_keys():
    """The reduction's reading, on the oracle's own tables: a cell counts when its key's level-two
    hash lands on it.  Over a built table those cells are exactly the n keys' cells (every fill copy
    sits where its key does not hash), so folding over them is folding over the input values."""
    import oracle
    from oracle import rounds, spec
    from paper_2508_11443_amd import workloads
    from tests import fkscheck
    for n, seed in [(1, 1), (9, 2), (5000, 3), (100003, 4)]:
        sigma = 0x51 + n
        keys = workloads.unique_u64(n, seed, dense_fraction=0.5)
        vals = np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        ref = oracle.build_u64(keys, vals, sigma)
        header, slots = ref.export()
        _, sizes_all, t_all = fkscheck.decode_header(header, n)
        sizes, tv = sizes_all[:n], t_all[:n]
        sq = sizes * sizes
        offs, owner = rounds.presum(sq), rounds.repiota(sq)
        ck, cv, _ = fkscheck.decode_cells(slots)
        S = ck.size
        local = np.arange(S) - offs[owner]
        own = np.zeros(S, bool)
        for t in np.unique(tv[owner]):
            sel = tv[owner] == t
            a0, a1, b = (int(x) for x in spec.level2_consts(sigma, ref.r, int(t)))
            own[sel] = rounds.hash_vec(a0, a1, b, ck[sel]) % sq[owner[sel]] == local[sel]
        assert own.sum() == n
        assert (np.sort(ck[own]) == np.sort(keys)).all()
        for op in (ov.VRED_SUM, ov.VRED_MIN, ov.VRED_MAX, ov.VRED_XOR):
            assert ov.reduce_values(cv[own], op) == ov.reduce_values(vals, op)
        if n >= 5000:
            # the table holds fill copies, and folding over every cell would count them
            assert (~own).sum() > 0
            assert ov.reduce_values(cv, ov.VRED_SUM) != ov.reduce_values(vals, ov.VRED_SUM)
