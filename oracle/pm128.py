"""Test oracle for PM+128: the PM+ construction over p = 2^128 + 51, the
smallest prime above 2^128 (Table "smallestprimes"), with 128-bit words.

THIS IS TEST INFRASTRUCTURE. Only the test suite and the CPU-baseline leg of
``bench.py`` may import it. The GPU library never imports, links or calls
anything here, and nothing here imports the library.

The paper gives only the prime for n = 128, so the rest follows the PM+32 /
PM+64 construction with n = 128 (readings fixed in the library's header
too):
  - words: the string, a byte 0x01, zero bytes to a multiple of 16, read as
    little-endian 128-bit words (end of Sec. 4);
  - f_j(s) = (b_j + sum_{i<128} a_{j,i} s_i) mod p (Eq. (1)); the tree of
    Algorithm 1 with leaves on the level-1 keys, at least one level, at most
    8 levels;
  - keys a in [1, p - kappa - 1] = [1, 2^128 - 50] with kappa = 2 (k - 1) =
    100 (k = 51), b in [0, 2^128); drawn from splitmix64 (seed) in storage
    order a[0][0..127], ..., a[7][..], b[0..7], each key from two draws, low
    64 bits first; an `a` draw outside the range is drawn again;
  - output h mod 2^128 (Sec. 5); there is no Sec. 7 mixer for n = 128, so
    the mixed and raw outputs coincide; FIELD gives h itself.
Python integers are exact, so every sum is reduced with a plain %.
"""
from __future__ import annotations

P128 = (1 << 128) + 51
K128 = 51
AMAX128 = (1 << 128) - 50  # p - kappa - 1, kappa = 2 (K128 - 1)
M1 = (1 << 64) - 1


def splitmix64(seed: int):
    """splitmix64 (Steele, Lea and Flood 2014) as an endless generator."""
    s = seed & M1
    while True:
        s = (s + 0x9E3779B97F4A7C15) & M1
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M1
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M1
        yield z ^ (z >> 31)


def expand_keys128(seed: int) -> tuple[list[list[int]], list[int]]:
    """(a[8][128], b[8]) as Python integers."""
    g = splitmix64(seed)

    def draw():
        lo = next(g)
        hi = next(g)
        return lo | (hi << 64)

    a = []
    for _ in range(8):
        row = []
        while len(row) < 128:
            v = draw()
            if 1 <= v <= AMAX128:
                row.append(v)
        a.append(row)
    b = [draw() for _ in range(8)]
    return a, b


def words(data: bytes) -> list[int]:
    """End of Sec. 4: append 0x01, pad with zeros to a multiple of 16 bytes,
    little-endian 128-bit words."""
    y = bytes(data) + b"\x01"
    y += b"\x00" * ((-len(y)) % 16)
    return [int.from_bytes(y[i:i + 16], "little") for i in range(0, len(y), 16)]


def tree(sigma: list[int], a, b, m: int = 128, lmax: int = 8) -> int:
    """Algorithm 1 as a do-while over levels: each level replaces the values by
    f_j of each run of m (a short last run counts the missing terms as 0)."""
    j = 0
    while True:
        if j == lmax:
            raise ValueError("more than lmax levels")
        nxt = []
        for c in range(0, len(sigma), m):
            s = b[j]
            for i, v in enumerate(sigma[c:c + m]):
                s += a[j][i] * v
            nxt.append(s % P128)
        sigma = nxt
        j += 1
        if len(sigma) == 1:
            return sigma[0]


def pm128(data: bytes, a, b, field: bool = False) -> int:
    """h (field) or h mod 2^128 (Sec. 5)."""
    h = tree(words(data), a, b)
    return h if field else h % (1 << 128)


def batch(buf, offsets, a, b, field: bool = False) -> list[int]:
    return [pm128(bytes(buf[offsets[i]:offsets[i + 1]]), a, b, field) for i in range(len(offsets) - 1)]


def key_table_u64(a, b):
    """The key table as 2064 uint64 (each entry lo, hi; a[8][128] then b[8])."""
    import numpy as np

    out = np.zeros(2 * (8 * 128 + 8), np.uint64)
    flat = [v for row in a for v in row] + list(b)
    for i, v in enumerate(flat):
        out[2 * i] = v & M1
        out[2 * i + 1] = v >> 64
    return out
