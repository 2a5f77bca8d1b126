"""Distinct byte strings with equal fingerprints, for tests of the rejection path.

Test infrastructure, CPU only.  Two strings of one length L = 4k have equal fingerprints
under base beta exactly when their little-endian 32-bit words w and w' satisfy
sum_i (w'_i - w_i) * beta^(k-1-i) == 0 (mod p), p = 2^61 - 1: Horner's rule expands
the fingerprint to L*beta^k + sum_i w_i * beta^(k-1-i).  The word differences d form a
lattice of determinant p in Z^k; for k = 4 its shortest vectors have entries near
p^(1/4) ~ 2^15, far inside the range of a 32-bit word, and the LLL reduction below
(Lenstra, Lenstra & Lovasz 1982, in exact rational arithmetic) finds one.
"""
from __future__ import annotations

from fractions import Fraction

P61 = (1 << 61) - 1


def _dot(u, v):
    return sum(a * b for a, b in zip(u, v))


def _gram_schmidt(B):
    Bs, mu = [], [[Fraction(0)] * len(B) for _ in B]
    for i, b in enumerate(B):
        v = [Fraction(x) for x in b]
        for j in range(i):
            mu[i][j] = _dot(b, Bs[j]) / _dot(Bs[j], Bs[j])
            v = [x - mu[i][j] * y for x, y in zip(v, Bs[j])]
        Bs.append(v)
    return Bs, mu


def lll(B, delta=Fraction(3, 4)):
    """LLL-reduced basis of the integer row vectors B (textbook form, exact)."""
    B = [list(b) for b in B]
    k = 1
    while k < len(B):
        Bs, mu = _gram_schmidt(B)
        for j in range(k - 1, -1, -1):
            q = round(mu[k][j])
            if q:
                B[k] = [x - q * y for x, y in zip(B[k], B[j])]
                Bs, mu = _gram_schmidt(B)
        if _dot(Bs[k], Bs[k]) >= (delta - mu[k][k - 1] ** 2) * _dot(Bs[k - 1], Bs[k - 1]):
            k += 1
        else:
            B[k], B[k - 1] = B[k - 1], B[k]
            k = max(k - 1, 1)
    return B


def word_difference(beta: int, k: int = 4):
    """A short non-zero d in Z^k with sum_i d_i * beta^(k-1-i) == 0 (mod p)."""
    basis = []
    for i in range(k - 1):
        row = [0] * k
        row[i] = 1
        row[k - 1] = (-pow(beta, k - 1 - i, P61)) % P61
        basis.append(row)
    basis.append([0] * (k - 1) + [P61])
    red = lll(basis)
    d = min((v for v in red if any(v)), key=lambda v: max(abs(x) for x in v))
    assert sum(x * pow(beta, k - 1 - i, P61) for i, x in enumerate(d)) % P61 == 0
    return d


def colliding_pair(beta: int, k: int = 4, fill: int = 0x61626364):
    """Two distinct strings of 4k bytes with equal fingerprints under beta."""
    d = word_difference(beta, k)
    assert max(abs(x) for x in d) < (1 << 30)
    w = [(fill + (1 << 31)) & 0xFFFFFFFF if x < 0 else fill for x in d]
    w2 = [a + x for a, x in zip(w, d)]
    assert all(0 <= v < (1 << 32) for v in w + w2)
    a = b"".join(v.to_bytes(4, "little") for v in w)
    b = b"".join(v.to_bytes(4, "little") for v in w2)
    assert a != b
    return a, b


def strings_with_collision(sigma: int, n_other: int, seed: int):
    """n_other random lowercase strings plus two strings of 16 bytes whose fingerprints are
    equal under the base of level-one attempt 0 of seed sigma (the first and the last key),
    as a CSR pair; the two are distinct from each other and from every other string."""
    import numpy as np

    from oracle import spec
    from paper_2508_11443_amd import workloads

    beta0 = spec.level1_consts(sigma, 0)[3]
    a, b = colliding_pair(beta0, fill=0x01020304)
    off, data = workloads.random_strings(n_other, seed, 4, 64)
    strings = [a] + workloads.from_csr(off, data) + [b]
    assert len(set(strings)) == len(strings)
    o, d = workloads.to_csr(strings)
    return np.asarray(o, np.int64), np.asarray(d, np.uint8), a, b
