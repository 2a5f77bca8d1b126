"""Pins for the oracle's primitives: the random stream, the hash family, the string
fingerprint.  None of these values comes from the oracle itself: they are a published
generator output, special cases that reduce to plain integer arithmetic, closed forms,
and statistical properties the paper requires of `random` and `hash` (Figure 1 text:
the constants must make `hash` a universal family)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import rounds, spec

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _impls():
    return [("c", oracle.splitmix, oracle.hash32, oracle.fingerprint),
            ("py", spec.splitmix, spec.hash32, spec.fingerprint)]


# ---- pin functions (reused by the mutation test) ----------------------------

def pin_splitmix_vector(splitmix):
    g = json.load(open(os.path.join(GOLD, "splitmix64_state0.json")))
    for i, hx in enumerate(g["outputs_hex"]):
        assert splitmix(g["seed"], i) == int(hx, 16), f"output {i}"


def pin_fin_inverse(splitmix):
    """fin is a bijection; undo it step by step and recover sigma + (i+1)*gamma."""
    def unxorshift(z, s):
        x = z
        for _ in range(64 // s + 1):
            x = z ^ (x >> s)
        return x & M64
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    rng = np.random.default_rng(11)
    for _ in range(200):
        sigma = int(rng.integers(0, np.iinfo(np.uint64).max, dtype=np.uint64, endpoint=True))
        i = int(rng.integers(0, 1 << 40))
        z = splitmix(sigma, i)
        z = unxorshift(z, 31)
        z = (z * inv2) & M64
        z = unxorshift(z, 27)
        z = (z * inv1) & M64
        z = unxorshift(z, 30)
        assert z == (sigma + (i + 1) * 0x9E3779B97F4A7C15) & M64


def pin_hash_special_cases(hash32):
    rng = np.random.default_rng(5)
    for _ in range(200):
        a0, a1, b = (int(v) for v in rng.integers(0, np.iinfo(np.uint64).max, size=3,
                                                  dtype=np.uint64, endpoint=True))
        # x = 0: only the additive constant survives
        assert hash32(a0, a1, b, 0) == b >> 32
        # x = 1: the low word multiplies a0
        assert hash32(a0, a1, b, 1) == ((a0 + b) % (1 << 64)) >> 32
        # x = 2^32: the high word multiplies a1
        assert hash32(a0, a1, b, 1 << 32) == ((a1 + b) % (1 << 64)) >> 32
        # with b = 0 and x < 2^32 the hash is the middle 32 bits of the 96-bit product a0*x
        x = int(rng.integers(0, 1 << 32))
        assert hash32(a0, a1, 0, x) == (a0 * x >> 32) % (1 << 32)
        # with b = 0 and only the high word set it is the middle bits of a1*hi
        assert hash32(a0, a1, 0, x << 32) == (a1 * x >> 32) % (1 << 32)
        assert 0 <= hash32(a0, a1, b, int(rng.integers(0, 1 << 63)) * 2 + 1) < (1 << 32)


def pin_hash_universal(hash_many, trials=20000, m=64):
    """For fixed distinct inputs the pair of hashes, reduced mod m, collides with
    probability close to 1/m over random constants (strong universality)."""
    rng = np.random.default_rng(9)
    A = rng.integers(0, np.iinfo(np.uint64).max, size=(trials, 3), dtype=np.uint64, endpoint=True)
    x = 0x0123456789ABCDEF
    for xp in (x ^ 1, x ^ (1 << 40), x + (1 << 32), x ^ 0xFFFF00000000):
        h1 = hash_many(A, x) % m
        h2 = hash_many(A, xp) % m
        rate = float(np.mean(h1 == h2))
        assert abs(rate - 1 / m) < 5 * np.sqrt((1 / m) / trials), (hex(xp), rate)
        # and each hash alone is uniform over the m residues
        counts = np.bincount(h1, minlength=m)
        chi2 = float(((counts - trials / m) ** 2 / (trials / m)).sum())
        assert chi2 < 130, chi2   # 63 degrees of freedom; p ~ 1e-6


def pin_fingerprint(fingerprint):
    rng = np.random.default_rng(3)
    p = spec.P61
    for _ in range(300):
        L = int(rng.integers(0, 70))
        data = bytes(rng.integers(0, 256, size=L, dtype=np.uint8))
        beta = int(rng.integers(1, p))
        w = [int.from_bytes((data[k:k + 4] + b"\0\0\0")[:4], "little") for k in range(0, L, 4)]
        mw = len(w)
        # closed form of the Horner recurrence: L*beta^m + sum_k w_k beta^(m-1-k)  (mod p)
        closed = (L * pow(beta, mw, p) + sum(wk * pow(beta, mw - 1 - k, p) for k, wk in enumerate(w))) % p
        assert fingerprint(data, beta) == closed
    assert fingerprint(b"", 12345) == 0
    # zero padding does not merge strings that differ only by trailing zero bytes
    assert fingerprint(b"ab", 77) != fingerprint(b"ab\0", 77)
    assert fingerprint(b"abcd", 77) != fingerprint(b"abcd\0\0\0\0", 77)


# ---- the tests ---------------------------------------------------------------

@pytest.mark.parametrize("name,splitmix,hash32,fingerprint", _impls())
def test_splitmix_published_vector(name, splitmix, hash32, fingerprint):
    pin_splitmix_vector(splitmix)


@pytest.mark.parametrize("name,splitmix,hash32,fingerprint", _impls())
def test_splitmix_inverse(name, splitmix, hash32, fingerprint):
    pin_fin_inverse(splitmix)


@pytest.mark.parametrize("name,splitmix,hash32,fingerprint", _impls())
def test_hash_special_cases(name, splitmix, hash32, fingerprint):
    pin_hash_special_cases(hash32)


def test_hash_universal_statistics():
    def many(A, x):
        return np.array([oracle.hash32(int(a[0]), int(a[1]), int(a[2]), x) for a in A[:4000]])
    pin_hash_universal(lambda A, x: many(A, x), trials=4000)

    def vec(A, x):
        xs = np.full(A.shape[0], x, np.uint64)
        lo, hi = xs & np.uint64(0xFFFFFFFF), xs >> np.uint64(32)
        with np.errstate(over="ignore"):
            return ((A[:, 0] * lo + A[:, 1] * hi + A[:, 2]) >> np.uint64(32)).astype(np.int64)
    pin_hash_universal(vec)


@pytest.mark.parametrize("name,splitmix,hash32,fingerprint", _impls())
def test_fingerprint_closed_form(name, splitmix, hash32, fingerprint):
    pin_fingerprint(fingerprint)


def test_c_and_python_agree_on_random_inputs():
    rng = np.random.default_rng(1)
    for _ in range(500):
        a0, a1, b, x, s = (int(v) for v in rng.integers(0, np.iinfo(np.uint64).max, size=5,
                                                       dtype=np.uint64, endpoint=True))
        assert oracle.hash32(a0, a1, b, x) == spec.hash32(a0, a1, b, x)
        i = int(rng.integers(0, 1 << 50))
        assert oracle.splitmix(s, i) == spec.splitmix(s, i)
    A = rng.integers(0, np.iinfo(np.uint64).max, size=(100, 3), dtype=np.uint64, endpoint=True)
    xs = rng.integers(0, np.iinfo(np.uint64).max, size=100, dtype=np.uint64, endpoint=True)
    for a, x in zip(A, xs):
        assert int(rounds.hash_vec(*(int(v) for v in a), np.array([x]))[0]) == spec.hash32(*(int(v) for v in a), int(x))


def test_attempt_constants_layout():
    sigma = 0xDEADBEEF
    for r in (0, 1, 5):
        a0, a1, b, beta = oracle.level1_consts(sigma, r)
        assert (a0, a1, b) == tuple(spec.splitmix(sigma, 772 * r + k) for k in range(3))
        assert 1 <= beta <= spec.P61 - 1
        assert (a0, a1, b, beta) == spec.level1_consts(sigma, r)
        for t in (0, 1, 63, 255):
            assert oracle.level2_consts(sigma, r, t) == spec.level2_consts(sigma, r, t)
            assert oracle.level2_consts(sigma, r, t)[0] == spec.splitmix(sigma, 772 * r + 4 + 3 * t)
    # batch seeds are the stream of the batch seed
    assert oracle.batch_seed(7, 3) == spec.splitmix(7, 3)


def test_vocabulary_golden():
    g = json.load(open(os.path.join(GOLD, "vocabulary.json")))
    assert rounds.sort([tuple(p) for p in g["sort"]["input"]]) == g["sort"]["output"]
    gb = g["groupby"]
    assert rounds.groupby(gb["m"], gb["idx"], gb["vals"]) == gb["output"]
    assert rounds.repiota(g["repiota"]["input"]).tolist() == g["repiota"]["output"]
    # presum is exclusive: it must give the first offset 0 and skip the last element
    assert rounds.presum([1, 4, 9]).tolist() == [0, 1, 5]
    # segor reduces each segment (sizes 2, 1, 3) to one flag
    assert rounds.segor([2, 1, 3], [0, 0, 1, 0, 0, 1]).tolist() == [False, True, True]
