"""Pins of the comparison-map oracle (sorted array + binary search, Eytzinger order;
the search structures the paper measures its hash maps against in Section 4).

The sorted layout is pinned by Python's own sort; the Eytzinger layout by the
binary-search-tree invariant on every node and by its in-order walk; lookups by
dictionary semantics.  A planted mistake (pre-order instead of in-order fill,
off-by-one child numbering) fails the invariants."""
import numpy as np
import pytest

import oracle


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    keys = np.unique(rng.integers(0, 2**64, size=2 * n + 8, dtype=np.uint64, endpoint=False))
    keys = rng.permutation(keys)[:n]
    vals = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    return keys, vals


def _inorder(a, i=1, out=None):
    out = [] if out is None else out
    if i <= len(a):
        _inorder(a, 2 * i, out)
        out.append(int(a[i - 1]))
        _inorder(a, 2 * i + 1, out)
    return out


def _subtree(a, i):
    if i > len(a):
        return []
    return [int(a[i - 1])] + _subtree(a, 2 * i) + _subtree(a, 2 * i + 1)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 7, 8, 9, 31, 32, 33, 100, 1000])
def test_sorted_layout_is_the_sorted_pairs(n):
    keys, vals = _pairs(n, 11 + n)
    sk, sv = oracle.search_build(keys, vals, 0)
    ref = sorted(zip(keys.tolist(), vals.tolist()))
    assert sk.tolist() == [k for k, _ in ref]
    assert sv.tolist() == [v for _, v in ref]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 15, 16, 17, 63, 64, 65, 200])
def test_eytzinger_is_a_search_tree_in_level_order(n):
    keys, vals = _pairs(n, 101 + n)
    ek, ev = oracle.search_build(keys, vals, 1)
    assert len(ek) == n
    # every node separates its two subtrees (the binary-search-tree invariant)
    for i in range(1, n + 1):
        left, right = _subtree(ek, 2 * i), _subtree(ek, 2 * i + 1)
        assert all(x < int(ek[i - 1]) for x in left)
        assert all(x > int(ek[i - 1]) for x in right)
    # the in-order walk gives back the sorted keys; values travel with their keys
    assert _inorder(ek) == sorted(keys.tolist())
    d = dict(zip(keys.tolist(), vals.tolist()))
    assert [d[int(k)] for k in ek] == ev.tolist()


def test_eytzinger_small_case_by_hand():
    # five keys: a complete tree with root 7, children 3 and 9, and 1, 5 under 3
    ek, ev = oracle.search_build(np.array([5, 3, 9, 1, 7], np.uint64), np.arange(5, dtype=np.uint32), 1)
    assert ek.tolist() == [7, 3, 9, 1, 5]
    assert ev.tolist() == [4, 1, 2, 3, 0]


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000, 4096])
def test_lookup_is_dictionary_semantics(layout, n):
    keys, vals = _pairs(n, 7 * n + layout)
    lk, lv = oracle.search_build(keys, vals, layout)
    rng = np.random.default_rng(5)
    absent = rng.integers(0, 2**64, size=600, dtype=np.uint64, endpoint=False)
    q = np.concatenate([keys[: min(n, 600)], absent, keys[: min(n, 10)] + np.uint64(1),
                        np.array([0, 2**64 - 1], np.uint64)])
    got_v, got_f = oracle.search_lookup(lk, lv, layout, q, missing=0xDEADBEEF)
    d = dict(zip(keys.tolist(), vals.tolist()))
    for x, v, f in zip(q.tolist(), got_v.tolist(), got_f.tolist()):
        assert f == (x in d)
        assert v == d.get(x, 0xDEADBEEF)


@pytest.mark.parametrize("layout", [0, 1])
def test_extreme_keys(layout):
    keys = np.array([0, 2**64 - 1, 1, 2**63], np.uint64)
    lk, lv = oracle.search_build(keys, np.arange(4, dtype=np.uint32), layout)
    v, f = oracle.search_lookup(lk, lv, layout, np.array([2**64 - 1, 0, 2**63, 2, 2**64 - 2], np.uint64))
    assert f.tolist() == [True, True, True, False, False]
    assert v.tolist()[:3] == [1, 0, 3]


@pytest.mark.parametrize("layout", [0, 1])
def test_duplicate_keys_are_rejected(layout):
    keys = np.array([4, 8, 15, 16, 8], np.uint64)
    with pytest.raises(oracle.OracleError) as e:
        oracle.search_build(keys, np.arange(5, dtype=np.uint32), layout)
    assert e.value.code == oracle.EDUPKEY


def test_planted_fill_mistakes_are_caught():
    """Pre-order fill, or children at 2i+1 / 2i+2 on a 1-based array, break the
    invariants the tests above check."""
    keys = sorted(_pairs(40, 3)[0].tolist())
    n = len(keys)

    def fill_preorder(i, it, out):
        if i <= n:
            out[i - 1] = next(it)
            fill_preorder(2 * i, it, out)
            fill_preorder(2 * i + 1, it, out)

    def fill_wrong_children(i, it, out):
        if i <= n:
            fill_wrong_children(2 * i + 1, it, out)
            out[i - 1] = next(it)
            fill_wrong_children(2 * i + 2, it, out)

    for bad_fill in (fill_preorder, fill_wrong_children):
        out = [None] * n
        try:
            bad_fill(1, iter(keys), out)
        except StopIteration:
            pass
        ok = None not in out and _inorder(out) == keys and all(
            all(x < out[i - 1] for x in _subtree(out, 2 * i)) for i in range(1, n + 1))
        assert not ok


def test_inorder_rank_helper_matches_the_recursive_fill():
    """The helper the GPU tests use at large sizes agrees with the oracle's
    recursive in-order fill on every node of every tree up to 300 nodes."""
    from tests import searchcheck
    for n in range(1, 301):
        keys = np.arange(n, dtype=np.uint64) * np.uint64(3) + np.uint64(5)
        ek, _ = oracle.search_build(keys, np.zeros(n, np.uint32), 1)
        for i in range(1, n + 1):
            assert int(ek[i - 1]) == int(keys[searchcheck.inorder_rank(i, n)])
