"""The fixed readings of the construction in pure Python integers.

Test infrastructure.  A second, independent statement of the primitives the C
oracle uses (SplitMix64 stream, multiply-shift hash, string fingerprint) and a
direct make_1 / make_2 (Section 2.3) for tiny inputs.  Python integers have no
overflow, so every reduction is written out explicitly.
"""
from __future__ import annotations

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1
GAMMA = 0x9E3779B97F4A7C15
STRIDE = 772          # stream entries per level-one attempt: 4 + 3 * 256
TMAX = 256
SMAX = 15
P61 = (1 << 61) - 1


def fin(z: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix(sigma: int, i: int) -> int:
    """Entry i of the stream seeded with sigma: state after i+1 steps of +gamma."""
    return fin(sigma + (i + 1) * GAMMA)


def hash32(a0: int, a1: int, b: int, x: int) -> int:
    """Thorup's vector multiply-shift: two 32-bit words of x, 64-bit arithmetic, top 32 bits."""
    lo, hi = x & M32, (x >> 32) & M32
    return ((a0 * lo + a1 * hi + b) & M64) >> 32


def level1_consts(sigma: int, r: int):
    base = r * STRIDE
    a0, a1, b = (splitmix(sigma, base + k) for k in range(3))
    beta = 1 + splitmix(sigma, base + 3) % (P61 - 1)
    return a0, a1, b, beta


def level2_consts(sigma: int, r: int, t: int):
    base = r * STRIDE + 4 + 3 * t
    return tuple(splitmix(sigma, base + k) for k in range(3))


def words32(data: bytes):
    """Little-endian 32-bit words of data, the last one zero padded."""
    out = []
    for k in range(0, len(data), 4):
        chunk = data[k:k + 4] + b"\0" * (4 - len(data[k:k + 4]))
        out.append(int.from_bytes(chunk, "little"))
    return out


def fingerprint(data: bytes, beta: int) -> int:
    """Horner evaluation of the word polynomial, seeded with the byte length, mod 2^61-1."""
    acc = len(data) % P61
    for w in words32(data):
        acc = (acc * beta + w) % P61
    return acc


def tag(c0, x: int) -> int:
    """Tag of the key of a one-key bucket: the top 8 bits of its trial-0 level-two hash."""
    return hash32(*c0, x) >> 24


def build_small(keys, vals, sigma, c=4, T=64, R=16):
    """make_1 / make_2 on Python lists (tiny n).  Returns a dict or raises ValueError(code)."""
    n = len(keys)
    if n == 0:
        return dict(n=0, S=0, r=0, sizes=[], t=[], tbyte=[], offsets=[0], cells=[])
    for r in range(R):
        a0, a1, b, _ = level1_consts(sigma, r)
        g = [hash32(a0, a1, b, x) % n for x in keys]
        sizes = [0] * n
        for j in g:
            sizes[j] += 1
        if max(sizes) > SMAX:
            continue
        offsets = [0]
        for s in sizes:
            offsets.append(offsets[-1] + s * s)
        S = offsets[-1]
        if S > c * n:
            continue
        groups = [[] for _ in range(n)]
        for i, j in enumerate(g):
            groups[j].append(i)
        C = [level2_consts(sigma, r, t) for t in range(T)]
        tj = [0] * n
        exhausted = dup = False
        for j in range(n):
            s = sizes[j]
            if s <= 1:
                continue
            for t in range(T):
                hs = [hash32(*C[t], keys[i]) % (s * s) for i in groups[j]]
                if len(set(hs)) == len(hs):
                    tj[j] = t
                    break
            else:
                exhausted = True
                ks = [keys[i] for i in groups[j]]
                dup = dup or len(set(ks)) < len(ks)
        if exhausted:
            if dup:
                raise ValueError("EDUPKEY")
            continue
        cells = [None] * S
        for i, x in enumerate(keys):
            j = g[i]
            s = sizes[j]
            p = offsets[j] + hash32(*C[tj[j]], x) % (s * s)
            cells[p] = (x, vals[i], 0)
        for j in range(n):
            lo, hi = offsets[j], offsets[j + 1]
            occ = [p for p in range(lo, hi) if cells[p] is not None]
            for p in range(lo, hi):
                if cells[p] is None:
                    cells[p] = cells[occ[0]]
        # the header byte of a bucket: its trial, or for a bucket of one key that key's tag
        tbyte = list(tj)
        for j in range(n):
            if sizes[j] == 1:
                tbyte[j] = tag(C[0], keys[groups[j][0]])
        return dict(n=n, S=S, r=r, sizes=sizes, t=tj, tbyte=tbyte, offsets=offsets, cells=cells,
                    a=(a0, a1, b), C=C)
    raise ValueError("EBUILD")


def pack_header(sizes, t):
    """The 16-byte group records for bucket sizes and header bytes (trial indices, and the
    tags of one-key buckets)."""
    n = len(sizes)
    out = bytearray()
    base = 0
    for g in range((n + 7) // 8):
        packed = 0
        tb = bytearray(8)
        gbase = base
        for k in range(8):
            j = 8 * g + k
            if j < n:
                packed |= sizes[j] << (4 * k)
                tb[k] = t[j]
                base += sizes[j] * sizes[j]
        out += gbase.to_bytes(4, "little") + packed.to_bytes(4, "little") + bytes(tb)
    return bytes(out)


def pack_cells(cells):
    out = bytearray()
    for key, val, aux in cells:
        out += key.to_bytes(8, "little") + val.to_bytes(4, "little") + aux.to_bytes(4, "little")
    return bytes(out)
