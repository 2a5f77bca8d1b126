"""Checks of a built table against what the paper fixes (Section 2.2) and the readings.

Given the keys, values, seed and an exported table (16-byte group headers and
16-byte cells, as either the oracle or the GPU library lays them out), verify:
  * bucket sizes are the histogram of g k = hash(const) k mod n (Section 2.2 shape);
  * group slot bases are the exclusive prefix sum of squared sizes (offsets);
  * total space S = sum of squares and S <= c*n (the level-one acceptance);
  * well-formed: h k lies in [0, S); collision free: h is injective on K;
  * every key's cell holds its key and value;
  * t of every bucket is the smallest trial index with no collision (make_2);
  * empty cells copy the lowest occupied cell of their bucket.
Vectorised with numpy so that it runs at sizes well past what pure Python can.
"""
from __future__ import annotations

import numpy as np

from oracle import rounds, spec


def decode_header(header: np.ndarray, n: int):
    """(group bases, bucket sizes, bucket trials).  A bucket of at most one key has trial 0:
    the byte of a one-key bucket is its key's tag (decode_tags)."""
    base, sizes, tbytes = _decode(header, n)
    return base, sizes, np.where(sizes >= 2, tbytes, 0)


def decode_tags(header: np.ndarray, n: int):
    """The raw per-bucket header bytes: the trial of a bucket of two or more keys, the tag of
    a one-key bucket's key, 0 for an empty bucket."""
    return _decode(header, n)[2]


def _decode(header, n):
    h = np.asarray(header, np.uint8).reshape(-1, 16)
    ng = (n + 7) // 8
    assert h.shape[0] == ng, (h.shape, ng)
    base = h[:, 0:4].copy().view(np.uint32).ravel().astype(np.int64)
    packed = h[:, 4:8].copy().view(np.uint32).ravel().astype(np.int64)
    shifts = 4 * np.arange(8, dtype=np.int64)
    sizes = ((packed[:, None] >> shifts[None, :]) & 15).ravel()
    tbytes = h[:, 8:16].astype(np.int64).ravel()
    return base, sizes, tbytes


def decode_cells(slots: np.ndarray):
    c = np.asarray(slots, np.uint8).reshape(-1, 16)
    keys = c[:, 0:8].copy().view(np.uint64).ravel()
    vals = c[:, 8:12].copy().view(np.uint32).ravel()
    aux = c[:, 12:16].copy().view(np.uint32).ravel()
    return keys, vals, aux


def check_table(keyv: np.ndarray, vals: np.ndarray, sigma: int, r: int, header, slots,
                c: int = 4, T: int = 64, aux=None, check_minimal: bool = True):
    """Raise AssertionError on the first violated property.  keyv are the hashed integers
    (the keys, or the string fingerprints under attempt r)."""
    keyv = np.asarray(keyv, np.uint64)
    n = keyv.size
    base, sizes_all, t_all = decode_header(header, n)
    raw_all = decode_tags(header, n)
    S = int(np.asarray(slots).size // 16)
    sizes, tv = sizes_all[:n], t_all[:n]
    assert (sizes_all[n:] == 0).all() and (raw_all[n:] == 0).all(), "padding buckets not zero"
    assert (raw_all[:n][sizes == 0] == 0).all(), "an empty bucket's header byte is not zero"
    a0, a1, b, _ = spec.level1_consts(sigma, r)
    g = rounds.hash_vec(a0, a1, b, keyv) % n
    counts = np.bincount(g, minlength=n)
    assert (counts == sizes).all(), "bucket sizes are not the level-one histogram"
    assert sizes.max(initial=0) <= spec.SMAX
    sq = sizes * sizes
    offs = rounds.presum(sq)
    gsum = np.add.reduceat(np.concatenate([sq, np.zeros((-n) % 8, np.int64)]),
                           np.arange(0, n + (-n) % 8, 8)) if n else np.zeros(0, np.int64)
    assert (base == rounds.presum(gsum)).all(), "group bases are not the exclusive prefix"
    assert S == int(sq.sum()), "table size is not the sum of squared sizes"
    assert S <= c * n, "space bound S <= c*n violated"
    assert (tv < T).all()
    # h k for every key
    C = np.array([spec.level2_consts(sigma, r, t) for t in range(T)], dtype=object)
    h = np.empty(n, np.int64)
    for t in np.unique(tv[g]):
        sel = tv[g] == t
        a0t, a1t, bt = (int(v) for v in C[t])
        h[sel] = rounds.hash_vec(a0t, a1t, bt, keyv[sel]) % sq[g[sel]]
    pos = offs[g] + h
    # the byte of a one-key bucket is its key's tag: the top 8 bits of the trial-0 hash
    one = sizes[g] == 1
    if one.any():
        a0t, a1t, bt = (int(v) for v in C[0])
        tags = (rounds.hash_vec(a0t, a1t, bt, keyv[one]) >> 24).astype(np.int64)
        assert (raw_all[g[one]] == tags).all(), "a one-key bucket's tag is not its key's"
    assert ((pos >= 0) & (pos < S)).all(), "not well formed"
    assert np.unique(pos).size == n, "not collision free"
    ck, cv, ca = decode_cells(slots)
    assert (ck[pos] == keyv).all(), "a key is not in its cell"
    assert (cv[pos] == np.asarray(vals, np.uint32)).all(), "a value is not in its key's cell"
    if aux is not None:
        assert (ca[pos] == np.asarray(aux, np.uint32)).all(), "aux word mismatch"
    # fill rule
    occupied = np.zeros(S, bool)
    occupied[pos] = True
    owner = rounds.repiota(sq)
    first = np.full(n, -1, np.int64)
    occ_idx = np.nonzero(occupied)[0]
    # lowest occupied cell per bucket: cells are in bucket order, so the first occupied
    # cell of each owner is found by taking unique owners over occupied cells
    u, at = np.unique(owner[occ_idx], return_index=True)
    first[u] = occ_idx[at]
    empty = np.nonzero(~occupied)[0]
    src = first[owner[empty]]
    assert (src >= 0).all()
    cells = np.asarray(slots, np.uint8).reshape(-1, 16)
    assert (cells[empty] == cells[src]).all(), "empty cell is not the bucket's lowest occupied cell"
    # minimality of t
    if check_minimal:
        big = np.nonzero((sizes >= 2) & (tv > 0))[0]
        if big.size:
            order = np.argsort(g, kind="stable")
            gs = g[order]
            start = np.searchsorted(gs, big)
            for t in range(int(tv[big].max())):
                live = big[tv[big] > t]
                if live.size == 0:
                    break
                st = np.searchsorted(gs, live)
                members = np.concatenate([order[s0:s0 + sizes[j]] for s0, j in zip(st, live)])
                owners = np.repeat(live, sizes[live])
                a0t, a1t, bt = (int(v) for v in C[t])
                hh = rounds.hash_vec(a0t, a1t, bt, keyv[members]) % sq[owners]
                cell = offs[owners] + hh
                # every live bucket must see a collision under trial t
                uniq = np.unique(cell)
                coll_owner = np.zeros(n, bool)
                _, cnt = np.unique(cell, return_counts=True)
                dupcells = uniq[cnt > 1]
                coll_owner[rounds.repiota(sq)[dupcells]] = True
                assert coll_owner[live].all(), f"t is not minimal (trial {t} was collision free)"
            del start
    return dict(n=n, S=S, sizes=sizes, t=tv, g=g, pos=pos)
