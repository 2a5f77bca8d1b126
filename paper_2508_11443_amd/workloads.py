"""Seeded synthetic workloads shaped like the paper's benchmarks (Section 4).

Uniform unique 64-bit keys with 32-bit values (the values are the key index),
lowercase byte strings, batches of independent maps and serving request
streams.  Only random numbers and set membership live here -- none of the
hash map's own arithmetic -- so the same arrays can feed both the GPU library
and the CPU checker.
"""
from __future__ import annotations

import numpy as np

U64_MAX = np.iinfo(np.uint64).max


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unique_keep_order(a: np.ndarray) -> np.ndarray:
    _, first = np.unique(a, return_index=True)
    first.sort()
    return a[first]


def _uniform_u64(rng, count):
    return rng.integers(0, U64_MAX, size=count, dtype=np.uint64, endpoint=True)


def unique_u64(n: int, seed: int, dense_fraction: float = 0.0) -> np.ndarray:
    """n distinct uint64 keys in random order.

    A ``dense_fraction`` of them is one run of consecutive integers starting at a
    random base; the rest are uniform and avoid that run.
    """
    rng = _rng(seed)
    nd = int(n * dense_fraction)
    nu = n - nd
    if nd:
        base = rng.integers(0, U64_MAX - np.uint64(nd), dtype=np.uint64, endpoint=True)
        dense = base + np.arange(nd, dtype=np.uint64)
        lo, hi = base, base + np.uint64(nd - 1)
    else:
        dense = np.zeros(0, np.uint64)
    out = np.zeros(0, np.uint64)
    while out.size < nu:
        need = nu - out.size
        cand = _uniform_u64(rng, need + need // 64 + 16)
        if nd:
            cand = cand[(cand < lo) | (cand > hi)]
        out = _unique_keep_order(np.concatenate([out, cand]))
    keys = np.concatenate([out[:nu], dense])
    rng.shuffle(keys)
    return keys


def absent_u64(keys_sorted: np.ndarray, count: int, rng) -> np.ndarray:
    """count uniform uint64 values that are not in keys_sorted (sorted array)."""
    out = np.zeros(0, np.uint64)
    while out.size < count:
        need = count - out.size
        cand = _uniform_u64(rng, need + 16)
        if keys_sorted.size:
            # membership through the candidates in sorted order (a cache-friendly search)
            order = np.argsort(cand, kind="stable")
            pos = np.searchsorted(keys_sorted, cand[order])
            pos = np.minimum(pos, keys_sorted.size - 1)
            present = np.empty(cand.size, bool)
            present[order] = keys_sorted[pos] == cand[order]
            cand = cand[~present]
        out = np.concatenate([out, cand])
    return out[:count]


def u64_queries(keys: np.ndarray, m: int, hit_fraction: float, seed: int, return_index: bool = False):
    """m queries: a hit_fraction of present keys (no repeats while possible) and uniform absent
    keys, in uniform random order.  Returns (queries, expected_found uint8), and with
    return_index also the position in `keys` of each present query (-1 for absent ones); the
    draws are the same either way."""
    rng = _rng(seed)
    nh = int(round(m * hit_fraction))
    if keys.size == 0:
        nh = 0
    if nh:
        if nh <= keys.size:
            idx = rng.permutation(keys.size)[:nh]
        else:
            idx = rng.integers(0, keys.size, size=nh)
        hits = keys[idx]
    else:
        hits = np.zeros(0, np.uint64)
    miss = absent_u64(np.sort(keys), m - nh, rng)
    q = np.concatenate([hits, miss])
    found = np.concatenate([np.ones(nh, np.uint8), np.zeros(m - nh, np.uint8)])
    perm = rng.permutation(m)
    if not return_index:
        return q[perm], found[perm]
    src = np.concatenate([idx.astype(np.int64) if nh else np.zeros(0, np.int64), np.full(m - nh, -1, np.int64)])
    return q[perm], found[perm], src[perm]


# ---- byte strings ----------------------------------------------------------

def random_strings(n: int, seed: int, min_len: int = 4, max_len: int = 64, unique: bool = True,
                   exclude=None):
    """n lowercase ASCII strings with lengths uniform in [min_len, max_len], as a CSR pair
    (int64 offsets[n+1], uint8 bytes), in random order.  With ``unique`` the strings are
    distinct.  ``exclude`` is a CSR pair (offsets, bytes) of strings none of them may equal."""
    rng = _rng(seed)
    lens = rng.integers(min_len, max_len, size=n, endpoint=True)
    ex_by_len = {}
    if exclude is not None:
        eoff, edata = exclude
        elens = eoff[1:] - eoff[:-1]
        for L in np.unique(elens):
            L = int(L)
            if L == 0:
                continue
            where = np.nonzero(elens == L)[0]
            rows = edata[eoff[where][:, None] + np.arange(L)[None, :]]
            ex_by_len[L] = np.unique(np.ascontiguousarray(rows).view(f"V{L}").ravel())
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    data = np.empty(int(offsets[-1]), np.uint8)
    for L in range(min_len, max_len + 1):
        where = np.nonzero(lens == L)[0]
        cnt = where.size
        if cnt == 0 or L == 0:
            continue
        got = np.zeros(0, f"V{L}")
        while got.size < cnt:
            need = cnt - got.size
            block = rng.integers(ord("a"), ord("z"), size=(need + need // 8 + 8, L), endpoint=True,
                                 dtype=np.uint8)
            cand = np.ascontiguousarray(block).view(f"V{L}").ravel()
            ex = ex_by_len.get(L)
            if ex is not None and ex.size:
                pos = np.minimum(np.searchsorted(ex, cand), ex.size - 1)
                cand = cand[ex[pos] != cand]
            got = np.concatenate([got, cand])
            if unique:
                got = _unique_keep_order(got)
        flat = np.ascontiguousarray(got[:cnt]).view(np.uint8).reshape(cnt, L)
        data[offsets[where][:, None] + np.arange(L)[None, :]] = flat
    return offsets, data


def gather_strings(offsets, data, idx):
    """CSR pair holding strings idx of (offsets, data), in that order."""
    idx = np.asarray(idx, np.int64)
    lens = offsets[idx + 1] - offsets[idx]
    out_off = np.zeros(idx.size + 1, np.int64)
    np.cumsum(lens, out=out_off[1:])
    total = int(out_off[-1])
    owner = np.repeat(np.arange(idx.size), lens)
    within = np.arange(total) - out_off[owner]
    out = data[offsets[idx][owner] + within] if total else np.zeros(0, np.uint8)
    return out_off, out


def concat_strings(a, b):
    aoff, adata = a
    boff, bdata = b
    off = np.concatenate([aoff, boff[1:] + aoff[-1]])
    return off, np.concatenate([adata, bdata])


def to_csr(strings):
    lens = np.fromiter((len(s) for s in strings), np.int64, count=len(strings))
    offsets = np.zeros(len(strings) + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    data = np.frombuffer(b"".join(strings), np.uint8).copy() if strings else np.zeros(0, np.uint8)
    return offsets, data


def from_csr(offsets, data):
    return [data[offsets[i]:offsets[i + 1]].tobytes() for i in range(offsets.size - 1)]


def string_queries(keys_off, keys_data, m: int, hit_fraction: float, seed: int,
                   min_len: int = 4, max_len: int = 64):
    """m string queries: hits drawn from the keys, misses from the same distribution but
    absent; uniform order.  Returns (offsets, bytes, expected_found, expected_index)."""
    rng = _rng(seed)
    n = keys_off.size - 1
    nh = int(round(m * hit_fraction)) if n else 0
    idx = rng.permutation(n)[:nh] if nh <= n else rng.integers(0, n, size=nh)
    hits = gather_strings(keys_off, keys_data, idx)
    misses = random_strings(m - nh, seed + 1, min_len, max_len, unique=False,
                            exclude=(keys_off, keys_data))
    allq = concat_strings(hits, misses)
    found = np.concatenate([np.ones(nh, np.uint8), np.zeros(m - nh, np.uint8)])
    index = np.concatenate([idx, np.full(m - nh, -1)]).astype(np.int64)
    perm = rng.permutation(m)
    off, data = gather_strings(allq[0], allq[1], perm)
    return off, data, found[perm], index[perm]


# ---- batches of maps -------------------------------------------------------

def batch_sizes(M: int, seed: int, lo: int = 16, hi: int = 1 << 16) -> np.ndarray:
    """Map sizes floor(exp(U[ln lo, ln hi])), i.e. log-uniform in [lo, hi]."""
    rng = _rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi), size=M)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def batch_u64(M: int, seed: int, lo: int = 16, hi: int = 1 << 16):
    """Keys of M independent maps concatenated: (keys, vals, map_offsets[M+1]).
    Keys are unique within each map; values are the index inside the map."""
    sizes = batch_sizes(M, seed, lo, hi)
    offsets = np.zeros(M + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    rng = _rng(seed + 1)
    keys = np.empty(offsets[-1], np.uint64)
    vals = np.empty(offsets[-1], np.uint32)
    total = int(offsets[-1])
    # one pool of unique keys, cut into the maps: keys are then unique within every map
    pool = np.zeros(0, np.uint64)
    while pool.size < total:
        pool = _unique_keep_order(np.concatenate([pool, _uniform_u64(rng, total - pool.size + 64)]))
    keys[:] = pool[:total]
    for m in range(M):
        vals[offsets[m]:offsets[m + 1]] = np.arange(sizes[m], dtype=np.uint32)
    return keys, vals, offsets


def batch_queries(keys, offsets, m: int, hit_fraction: float, seed: int):
    """(map_ids u32, queries u64, expected_found u8, expected_value u32) spread uniformly over
    the maps; a hit_fraction are keys of the chosen map, the rest keys absent from it."""
    rng = _rng(seed)
    M = offsets.size - 1
    ids = rng.integers(0, M, size=m).astype(np.uint32)
    sizes = (offsets[1:] - offsets[:-1])
    hit = (rng.random(m) < hit_fraction) & (sizes[ids] > 0)
    pick = (rng.random(m) * sizes[ids]).astype(np.int64)
    q = np.empty(m, np.uint64)
    q[hit] = keys[offsets[ids[hit]] + pick[hit]]
    all_sorted = np.sort(keys)
    q[~hit] = absent_u64(all_sorted, int((~hit).sum()), rng)
    exp_val = np.where(hit, pick, 0).astype(np.uint32)
    return ids, q, hit.astype(np.uint8), exp_val


# ---- serving request streams -----------------------------------------------

def serving_requests(count: int, rate_per_s: float, seed: int, build_fraction: float = 0.2,
                     build_lo: int = 1 << 10, build_hi: int = 1 << 24,
                     lookup_lo: int = 1 << 8, lookup_hi: int = 1 << 20):
    """A Poisson stream: list of dicts {t (s), kind ('build'|'lookup'), size, seed}."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    kinds = rng.random(count) < build_fraction
    out = []
    for i in range(count):
        if kinds[i]:
            size = int(np.floor(np.exp(rng.uniform(np.log(build_lo), np.log(build_hi)))))
            out.append(dict(t=float(t[i]), kind="build", size=size, seed=int(rng.integers(1 << 62))))
        else:
            size = int(np.floor(np.exp(rng.uniform(np.log(lookup_lo), np.log(lookup_hi)))))
            out.append(dict(t=float(t[i]), kind="lookup", size=size, seed=int(rng.integers(1 << 62)),
                            pick=float(rng.random())))
    return out


# ---- counter-indexed unique keys (device or host) ----------------------------------
# A fixed invertible mixer of 64-bit integers (odd multiplications and xor-shifts are
# bijections mod 2^64), so distinct indices give distinct keys without a uniqueness
# pass.  Used to make large serving workloads quickly on the GPU.  It is unrelated to
# the hash map's own arithmetic.

_MIX_A = 0xD6E8FEB86659FD93
_MIX_B = 0xA0761D6478BD642F


def mix_keys_np(idx):
    x = np.asarray(idx, np.uint64)
    with np.errstate(over="ignore"):
        x = x * np.uint64(_MIX_A)
        x ^= x >> np.uint64(32)
        x = x * np.uint64(_MIX_B)
        x ^= x >> np.uint64(29)
    return x


def _srl(t, s):
    import torch
    return (t >> s) & torch.tensor((1 << (64 - s)) - 1, dtype=torch.int64, device=t.device)


def mix_keys_torch(idx):
    """Same keys as mix_keys_np, computed on the tensor's device (int64 holding uint64 bits)."""
    import torch
    a = torch.tensor(_MIX_A - (1 << 64), dtype=torch.int64, device=idx.device)
    b = torch.tensor(_MIX_B - (1 << 64), dtype=torch.int64, device=idx.device)
    x = idx.to(torch.int64) * a
    x = x ^ _srl(x, 32)
    x = x * b
    x = x ^ _srl(x, 29)
    return x
