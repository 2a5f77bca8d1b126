"""Keys whose level-two search needs a late trial, for tests of the trials the final pass does
not keep in LDS.

Test infrastructure, CPU only.  For seed sigma and level-one attempt 0, bucket 0 of an n-key map
receives exactly s chosen keys such that each of the trials 0 .. t_min-1 maps two of them to the
same one of the bucket's s^2 cells (the birthday bound gives a random set of s keys such a
collision in a trial with probability about 0.4, so t_min consecutive ones almost never happen by
chance).  The keys are picked greedily from random candidates that hash to bucket 0: each
addition is the candidate that creates collisions in the most trials not yet covered.  The
other n - s keys are random keys of other buckets.  The hashes are the fixed readings' (the
multiply-shift hash of the SplitMix64 stream's triples), computed here on numpy arrays and
checked against the oracle's tables by the tests that use them.
"""
from __future__ import annotations

import numpy as np

from oracle import spec

M32 = np.uint64(0xFFFFFFFF)


def _hash32(c, x):
    """The multiply-shift hash of the uint64 array x under triple c (arithmetic mod 2^64)."""
    a0, a1, b = (np.uint64(v) for v in c)
    with np.errstate(over="ignore"):
        return ((a0 * (x & M32) + a1 * (x >> np.uint64(32)) + b) >> np.uint64(32)).astype(np.uint64)


def keys_with_late_trial(sigma: int, n: int, s: int, t_min: int = 16, rng_seed: int = 1,
                         pool: int = 6000, tries: int = 20) -> np.ndarray:
    """n distinct uint64 keys; bucket 0 of attempt 0 holds s of them, none of trials
    0 .. t_min-1 separates them.  Raises RuntimeError if the greedy choice fails tries times."""
    assert 2 <= s <= spec.SMAX and n > s
    rng = np.random.default_rng(rng_seed)
    a0, a1, b, _ = spec.level1_consts(sigma, 0)
    l1 = (a0, a1, b)
    C = [spec.level2_consts(sigma, 0, t) for t in range(t_min)]
    cells = np.uint64(s * s)
    # candidates of bucket 0
    cand = []
    have = 0
    while have < pool:
        x = rng.integers(0, 1 << 64, size=1 << 20, dtype=np.uint64)
        x = x[_hash32(l1, x) % np.uint64(n) == 0]
        cand.append(x)
        have += x.size
    cand = np.unique(np.concatenate(cand))
    H = np.stack([_hash32(c, cand) % cells for c in C], axis=1)   # candidate x trial -> cell
    for attempt in range(tries):
        chosen = [int(rng.integers(cand.size))]
        while len(chosen) < s:
            uncovered = np.array([len(set(H[chosen, t].tolist())) == len(chosen) for t in range(t_min)])
            gain = np.zeros(cand.size, np.int64)
            for t in np.flatnonzero(uncovered):
                gain += np.isin(H[:, t], H[chosen, t])
            gain[chosen] = -1
            chosen.append(int(np.argmax(gain)))
        if all(len(set(H[chosen, t].tolist())) < s for t in range(t_min)):
            break
    else:
        raise RuntimeError("no key set found")
    bucket = cand[chosen]
    # the other keys: random keys of the other buckets
    rest = []
    need = n - s
    while need > 0:
        x = rng.integers(0, 1 << 64, size=2 * need + 64, dtype=np.uint64)
        x = x[_hash32(l1, x) % np.uint64(n) != 0]
        x = np.setdiff1d(np.unique(x), bucket)
        rest.append(x[:need])
        need -= rest[-1].size
    keys = np.concatenate([bucket] + rest)
    assert np.unique(keys).size == n
    return rng.permutation(keys)
