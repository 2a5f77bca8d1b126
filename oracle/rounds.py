"""The sortless flattened construction (Section 2.5) in numpy.  Test infrastructure.

Written from the paper's data-parallel vocabulary (Figure 1) so that a reader can
set it beside the derivation: presum, hist, repiota, segor, partition, filter,
scatter.  Readings taken where the text is open:
  * presum is the exclusive prefix sum;
  * segor reduces each segment to one flag (the collision flag of a bucket);
  * segrandom hands every remaining bucket the same triple in a round: round t
    uses level-two triple t of the attempt, so a bucket that first becomes
    collision free in round t ends with t -- the same t as make_2's first
    success;
  * the flat cell space of a round is the sum of the squared sizes;
  * empty buckets get trial index 0.
"""
from __future__ import annotations

import numpy as np

from . import spec

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


# ---- Figure 1 vocabulary ---------------------------------------------------

def presum(a):
    """Exclusive prefix sum."""
    a = np.asarray(a, dtype=np.int64)
    out = np.zeros(a.size, np.int64)
    if a.size > 1:
        np.cumsum(a[:-1], out=out[1:])
    return out


def hist(nbins, idx, vals):
    out = np.zeros(nbins, np.int64)
    np.add.at(out, np.asarray(idx, np.int64), np.asarray(vals, np.int64))
    return out


def repiota(a):
    a = np.asarray(a, np.int64)
    return np.repeat(np.arange(a.size, dtype=np.int64), a)


def segor(shape, flags):
    """One flag per segment: the logical or of the segment's flags."""
    shape = np.asarray(shape, np.int64)
    seg = repiota(shape)
    out = np.zeros(shape.size, bool)
    np.logical_or.at(out, seg, np.asarray(flags, bool))
    return out


def partition(pred, arr):
    pred = np.asarray(pred, bool)
    return arr[pred], arr[~pred]


def filter_(pred, arr):
    return arr[np.asarray(pred, bool)]


def scatter(dest, idx, vals):
    out = np.array(dest, copy=True)
    out[np.asarray(idx, np.int64)] = vals
    return out


def groupby(m, idx, vals):
    out = [[] for _ in range(m)]
    for i, v in zip(idx, vals):
        out[i].append(v)
    return out


def sort(pairs):
    """Stable sort by the first component, keeping the second."""
    order = sorted(range(len(pairs)), key=lambda i: pairs[i][0])
    return [pairs[i][1] for i in order]


# ---- hashing on arrays -----------------------------------------------------

def hash_vec(a0, a1, b, x):
    """Multiply-shift over a uint64 array; numpy uint64 arithmetic wraps mod 2^64."""
    x = np.asarray(x, np.uint64)
    lo = x & _M32
    hi = x >> _S32
    with np.errstate(over="ignore"):
        acc = np.uint64(a0) * lo + np.uint64(a1) * hi + np.uint64(b)
    return (acc >> _S32).astype(np.int64)


# ---- the construction ------------------------------------------------------

def seghashes(shape, triple, okeys_o, okeys_k):
    offsets = presum(shape * shape)
    o2 = offsets[okeys_o]
    s = shape[okeys_o]
    return o2 + hash_vec(*triple, okeys_k) % (s * s)


def segcollisions(shape, hashes):
    sshape = shape * shape
    flat = int(sshape.sum())
    counts = hist(flat, hashes, np.ones(hashes.size, np.int64))
    return segor(sshape, counts > 1)


def segmake2(shape, keys, hashes, triples):
    """Returns (t per bucket, exhausted bucket indices)."""
    n = shape.size
    offsets = presum(shape != 0)
    okeys_o = offsets[hashes]
    okeys_k = np.asarray(keys, np.uint64)
    idx = np.arange(n, dtype=np.int64)
    keep = shape != 0
    ish_i, ish_s = idx[keep], shape[keep]
    done_i, done_t = [], []
    for rnd, triple in enumerate(triples):
        if okeys_k.size == 0:
            break
        hs = seghashes(ish_s, triple, okeys_o, okeys_k)
        coll = segcollisions(ish_s, hs)
        # segresult: partition bucket positions by collision
        notdone, done = partition(coll, np.arange(ish_s.size))
        done_i.append(ish_i[done])
        done_t.append(np.full(done.size, rnd, np.int64))
        # keep the keys of colliding buckets and re-index them
        keep_k = coll[okeys_o]
        okeys_k = filter_(keep_k, okeys_k)
        okeys_o = filter_(keep_k, okeys_o)
        reidx = presum(coll.astype(np.int64))
        okeys_o = reidx[okeys_o]
        ish_i, ish_s = ish_i[notdone], ish_s[notdone]
    t = np.zeros(n, np.int64)
    if done_i:
        t = scatter(t, np.concatenate(done_i), np.concatenate(done_t))
    return t, ish_i


def make1(keys, sigma, r, T):
    """One level-one attempt: (bucket of every key, bucket sizes, t per bucket, exhausted)."""
    keys = np.asarray(keys, np.uint64)
    n = keys.size
    a0, a1, b, _ = spec.level1_consts(sigma, r)
    hashes = hash_vec(a0, a1, b, keys) % n
    shape = hist(n, hashes, np.ones(n, np.int64))
    triples = [spec.level2_consts(sigma, r, t) for t in range(T)]
    t, exhausted = segmake2(shape, keys, hashes, triples)
    return hashes, shape, t, exhausted
