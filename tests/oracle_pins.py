"""Pins that tie the CPU oracle to facts fixed by the paper and by plain
mathematics, rather than to a second copy of its own formula.

Each ``pin_*`` function takes a loaded oracle and raises AssertionError when
the oracle disagrees. ``test_oracle_pins.py`` runs them on the real oracle;
``test_oracle_mutants.py`` runs them on copies of the oracle with planted
mistakes and checks that every mistake trips at least one pin.

What pins what:
  primes / single product   Table "smallestprimes", Sec. 5: p = 2^n + k is the
                            smallest prime above 2^n (sympy), and one product
                            c * x mod p is plain integer arithmetic.
  word formation            end of Sec. 4: little-endian words of
                            bytes || 0x01 || zeros, read with int.from_bytes,
                            selected one at a time by unit keys.
  tree shape                Algorithm 1 and Fig. 1 (m = 4 worked example), and
                            unit keys at every level that select one leaf word.
  level count               Algorithm 1 with at least one level: the smallest
                            L >= 1 with m^L >= number of padded words.
  linearity                 Eq. (1) is affine in each level's keys over F_p.
  full field elements       Sec. 6.1: values above the first level stay in
                            [0, p) and are not cut to one word.
  mixers                    Sec. 7 printed constants (hand values) and
                            invertibility (an inverse written here).
  regularity                Lemma 9: with all other words fixed, the field
                            output is a bijection of the swept word (2^20
                            contiguous values across the wrap past p); the
                            n-bit output has at most 2 preimages, exactly k
                            of them twice when a_r = 1 (Lemma 8).
  single-key collisions     Lemma 9 / Sec. 5 bound: over one key a_r the
                            field outputs of a fixed pair collide at exactly
                            the t the modular inverse predicts, n-bit outputs
                            at no more than three predicted t.
  key expansion             published splitmix64 outputs, key ranges of
                            Eq. (1) with kappa from Table "parameters".
"""
from __future__ import annotations

import os

import numpy as np
import sympy

import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

P32 = int(sympy.nextprime(1 << 32))
P64 = int(sympy.nextprime(1 << 64))
AMAX32 = P32 - 28 - 1  # largest key in (0, p - kappa), kappa = 28
AMAX64 = P64 - 24 - 1  # kappa = 24
M = 128


def _gold_lines(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _padded(data: bytes, W: int) -> bytes:
    y = data + b"\x01"
    return y + b"\x00" * ((-len(y)) % W)


def _words(data: bytes, W: int) -> list[int]:
    y = _padded(data, W)
    return [int.from_bytes(y[i:i + W], "little") for i in range(0, len(y), W)]


def _keys(wide: bool, a=None, b=None):
    """Key table with the given level-major a[8][128] and b[8] (zeros default)."""
    k = np.zeros(1032, dtype=np.uint64 if wide else np.uint32)
    if a is not None:
        k[:1024] = np.asarray(a, dtype=k.dtype).reshape(-1)
    if b is not None:
        k[1024:] = np.asarray(b, dtype=k.dtype)
    return k


def _unit(wide: bool, picks: dict, b=None):
    """a[level][index] = value for (level, index) -> value in picks."""
    a = np.zeros((8, M), dtype=np.uint64 if wide else np.uint32)
    for (lvl, idx), v in picks.items():
        a[lvl, idx] = v
    return _keys(wide, a, b)


def _h(o, wide, data, keys, mode=O.FIELD):
    return (o.pm64 if wide else o.pm32)(data, keys, mode)


# ---------------------------------------------------------------------------
def pin_prime_table(o):
    """Table smallestprimes: each printed prime is prime and minimal; the
    fixture also carries the PM+ parameters of Table parameters."""
    for n, k in ((int(a), int(b)) for a, b in _gold_lines("smallest_primes.txt")):
        assert sympy.isprime((1 << n) + k)
        assert int(sympy.nextprime(1 << n)) == (1 << n) + k
    for n, k, kappa, m, L in ((int(x) for x in row) for row in _gold_lines("parameters.txt")):
        assert kappa == 2 * (k - 1) and m == 128 and L == 8
        p = (1 << n) + k
        # largest key times largest field element fits in two words (Sec. 6.1)
        assert (p - kappa - 1) * (p - 1) < 1 << (2 * n)


def pin_single_product(o):
    """One non-zero key a_{1,0} = c and word sigma_0 = x: h = c * x mod p."""
    rng = np.random.default_rng(11)
    for wide, p, amax, W in ((False, P32, AMAX32, 4), (True, P64, AMAX64, 8)):
        cases = [(1, 0), (1, 1), (amax, (1 << 8 * W) - 1), (2, (1 << 8 * W) - 1), (1 << (8 * W - 1), 4)]
        for _ in range(20):
            cases.append((int(rng.integers(1, amax, dtype=np.uint64)) if not wide else
                          int.from_bytes(rng.bytes(8), "little") % amax + 1,
                          int.from_bytes(rng.bytes(W), "little")))
        for c, x in cases:
            keys = _unit(wide, {(0, 0): c})
            h, L = _h(o, wide, x.to_bytes(W, "little"), keys)
            assert L == 1
            assert h == (c * x) % p, (wide, c, x, h)


def pin_word_formation(o):
    """Unit key e_r at level 1 returns padded word r (little-endian) for every
    word position of one-block strings, including the pad word."""
    rng = np.random.default_rng(12)
    for wide, W in ((False, 4), (True, 8)):
        for ln in [0, 1, 2, W - 1, W, W + 1, 2 * W - 1, 2 * W, 37, 100, M * W - W - 1, M * W - W]:
            data = rng.bytes(ln)
            words = _words(data, W)
            assert len(words) == ln // W + 1
            for r in sorted({0, 1, len(words) - 2, len(words) - 1, len(words), M - 1} & set(range(M))):
                h, L = _h(o, wide, data, _unit(wide, {(0, r): 1}))
                assert L == 1
                want = words[r] if r < len(words) else 0
                assert h == want, (wide, ln, r, h, want)


def pin_constant_term(o):
    """With all a = 0: one level gives b_1; two levels with a_2 = all ones give
    (number of level-1 blocks * b_1 + b_2) mod p."""
    for wide, p, W in ((False, P32, 4), (True, P64, 8)):
        top = (1 << 8 * W) - 1
        b = [top - j for j in range(8)]
        h, L = _h(o, wide, b"abc", _keys(wide, None, b))
        assert (h, L) == (b[0], 1)
        a = np.zeros((8, M), dtype=np.uint64)
        a[1, :] = 1
        for ln in (M * W - 1 - (W - 1), M * W, 5 * M * W + 3, M * M * W - W - 1):
            nwords = ln // W + 1
            blocks = -(-nwords // M)
            h, L = _h(o, wide, bytes(ln), _keys(wide, a, b))
            assert L == (1 if blocks == 1 else 2)
            want = b[0] if blocks == 1 else (blocks * b[0] + b[1]) % p
            assert h == want, (wide, ln, h, want)


def pin_checksum(o):
    """a_1 = all ones, b = 0: the sum of the padded words mod p; with the
    largest key it is (amax * sum) mod p. All-0xff data stresses carries."""
    rng = np.random.default_rng(13)
    for wide, p, amax, W in ((False, P32, AMAX32, 4), (True, P64, AMAX64, 8)):
        for data in (b"\xff" * (M * W - W), rng.bytes(M * W - W - 3), rng.bytes(17)):
            words = _words(data, W)
            for c in (1, amax):
                a = np.zeros((8, M), dtype=np.uint64)
                a[0, :] = c
                h, _ = _h(o, wide, data, _keys(wide, a))
                assert h == (c * sum(words)) % p


def pin_tree_projection(o):
    """Unit keys at levels 1..3 select leaf word 128*(128*d + c) + r of strings
    with two and three levels (Algorithm 1: leaves use level-1 keys, block c
    of level j feeds position c mod 128 of level j+1)."""
    rng = np.random.default_rng(14)
    for wide, W in ((False, 4), (True, 8)):
        for ln in (M * W, M * W + 1, 3 * M * W - 5, M * M * W - W - 1):
            data = rng.bytes(ln)
            words = _words(data, W)
            n = len(words)
            assert n > M
            for idx in {0, 1, M - 1, M, n - 1, n - 2, n // 2}:
                c, r = divmod(idx, M)
                h, L = _h(o, wide, data, _unit(wide, {(0, r): 1, (1, c): 1}))
                assert L == 2 and h == words[idx], (wide, ln, idx)
        ln = M * M * W + 2 * M * W + 7  # three levels
        data = rng.bytes(ln)
        words = _words(data, W)
        n = len(words)
        for idx in (0, M * M - 1, M * M, n - 1, M * M + M + 3):
            d, rest = divmod(idx, M * M)
            c, r = divmod(rest, M)
            h, L = _h(o, wide, data, _unit(wide, {(0, r): 1, (1, c): 1, (2, d): 1}))
            assert L == 3 and h == words[idx], (wide, idx)


def pin_level_count(o):
    """Levels used = the smallest L >= 1 with 128^L >= N', N' = floor(len/W)+1."""
    for wide, W in ((False, 4), (True, 8)):
        for nwords in (1, 2, M - 1, M, M + 1, M * M, M * M + 1):
            for extra in (0, W - 1):
                ln = (nwords - 1) * W + extra
                L = 1
                while M ** L < nwords:
                    L += 1
                _, got = _h(o, wide, bytes(ln), _keys(wide))
                assert got == L, (wide, ln, got, L)


def pin_fig1(o):
    """Fig. 1 worked example with m = 4 and one character per word:
    "ab" -> f1(a,b,1,0); "abcde" -> f2(f1(a,b,c,d), f1(e,1,0,0), 0, 0).
    Keys are positional weights so that each f is a readable base-2^7 /
    base-2^28 number well below p, and the pictured composition can be read
    back from the output."""
    A, B, C, D, E = (ord(ch) for ch in "abcde")
    wt1 = [1, 1 << 7, 1 << 14, 1 << 21]
    wt2 = [1, 1 << 28, 0, 0]  # the pictured level 2 has two live inputs

    def f1(w):
        return sum(x * y for x, y in zip(w, wt1))

    for wide, p in ((False, P32), (True, P64)):
        words_fn = o.words64 if wide else o.words32
        a = np.zeros((3, 4), dtype=np.uint64)
        a[0] = wt1
        a[1] = wt2
        b = np.zeros(3, dtype=np.uint64)
        h, L = words_fn([A, B, 1], a, b, 4, 3)
        assert (h, L) == (f1([A, B, 1, 0]), 1)
        h, L = words_fn([A, B, C, D, E, 1], a, b, 4, 3)
        want = (f1([A, B, C, D]) + (1 << 28) * f1([E, 1, 0, 0])) % p
        assert L == 2 and h == want, (wide, h, want)


def pin_linearity(o):
    """Affine in each level's keys (Eq. (1) over F_p): for key vectors x, y
    and step d at one level, F(x+d) - F(x) == F(y+d) - F(y) (mod p), and at
    one level F(a+d, b) == F(a, b) + F(d, 0) (mod p)."""
    rng = np.random.default_rng(15)
    for wide, p, amax, W in ((False, P32, AMAX32, 4), (True, P64, AMAX64, 8)):
        def rnd(n, hi):
            return np.array([int.from_bytes(rng.bytes(8), "little") % hi for _ in range(n)], dtype=np.uint64)

        half = amax // 2
        base_a = rnd(8 * M, half).reshape(8, M)
        base_b = rnd(8, 1 << 8 * W)
        data1 = rng.bytes(300)
        fa = _h(o, wide, data1, _keys(wide, base_a, base_b))[0]
        d = np.zeros((8, M), dtype=np.uint64)
        d[0] = rnd(M, half)
        fad = _h(o, wide, data1, _keys(wide, base_a + d, base_b))[0]
        fd0 = _h(o, wide, data1, _keys(wide, d, np.zeros(8)))[0]
        assert (fad - fa - fd0) % p == 0
        data2 = rng.bytes(M * M * W + 1000)  # three levels
        for lvl in (0, 1, 2):
            d = np.zeros((8, M), dtype=np.uint64)
            d[lvl] = rnd(M, half)
            y = base_a.copy()
            y[lvl] = rnd(M, half)
            f = [_h(o, wide, data2, _keys(wide, k, base_b))[0] for k in (base_a, base_a + d, y, y + d)]
            assert (f[1] - f[0] - (f[3] - f[2])) % p == 0, (wide, lvl)


def pin_full_field_values(o):
    """Sec. 6.1: values above the first level are field elements that can
    exceed one word. Level-1 value b_1 + 1*5 = 2^n + 4 < p must reach the
    root unchanged through a level-2 projection."""
    for wide, W in ((False, 4), (True, 8)):
        top = (1 << 8 * W) - 1
        keys = _unit(wide, {(0, 0): 5, (1, 0): 1}, [top] + [0] * 7)
        data = (1).to_bytes(W, "little") + bytes(M * W)
        h, L = _h(o, wide, data, keys)
        assert L == 2 and h == top + 5, (wide, h)
        raw, _ = _h(o, wide, data, keys, O.RAW)
        assert raw == 4


def pin_output_modes(o):
    """RAW is h mod 2^n and MIXED is the Sec. 7 mixer of RAW."""
    rng = np.random.default_rng(16)
    k32, k64 = o.expand_keys32(5), o.expand_keys64(6)
    for ln in (0, 3, 64, 1000, 70000):
        data = rng.bytes(ln)
        f, _ = o.pm32(data, k32, O.FIELD)
        assert o.pm32(data, k32, O.RAW)[0] == f % (1 << 32)
        assert o.pm32(data, k32, O.MIXED)[0] == o.mix32(f % (1 << 32))
        f, _ = o.pm64(data, k64, O.FIELD)
        assert o.pm64(data, k64, O.RAW)[0] == f % (1 << 64)
        assert o.pm64(data, k64, O.MIXED)[0] == o.mix64(f % (1 << 64))


def _inv_xorshift(z, s, bits):
    x = z
    for _ in range(bits // s + 1):
        x = z ^ (x >> s)
    return x & ((1 << bits) - 1)


def pin_mixers(o):
    """Hand values from the printed constants, and invertibility (Sec. 7
    claims the mixers are bijections): undo them with an inverse written
    here (xorshift inverse, modular inverse of the odd multiplier)."""
    for bits, x, want in ((int(a), int(b, 16), int(c, 16)) for a, b, c in _gold_lines("mixers.txt")):
        got = o.mix32(x) if bits == 32 else o.mix64(x)
        assert got == want, (bits, x, got, want)
    rng = np.random.default_rng(17)
    for bits, mix, mul, s1, s2 in ((32, o.mix32, 0xab3be54f, 13, 16), (64, o.mix64, 0xc4ceb9fe1a85ec53, 33, 33)):
        inv = pow(mul, -1, 1 << bits)
        for _ in range(200):
            z = int.from_bytes(rng.bytes(bits // 8), "little")
            y = mix(z)
            back = _inv_xorshift((_inv_xorshift(y, s2, bits) * inv) % (1 << bits), s1, bits)
            assert back == z


def _sweep_word(o, wide, base: bytes, r: int, lo: int, n: int, keys, mode=O.FIELD):
    """Outputs of the oracle for n copies of base whose word r takes the
    values lo, lo + 1, ..., lo + n - 1 (one batch call: every copy is hashed
    by the oracle in full)."""
    W = 8 if wide else 4
    L = len(base)
    vals = np.arange(n, dtype=np.uint64) + np.uint64(lo)
    buf = np.tile(np.frombuffer(base, np.uint8), n).reshape(n, L)
    buf[:, r * W:(r + 1) * W] = vals.astype("<u8").view(np.uint8).reshape(n, 8)[:, :W]
    off = np.arange(n + 1, dtype=np.int64) * L
    out = o.batch(wide, buf.reshape(-1), off, keys, mode, nthreads=os.cpu_count() or 1)
    if wide and mode == O.FIELD:
        return [int(a) | (int(b) << 64) for a, b in out]
    return [int(v) for v in out]


def _preimage_counts(f, n):
    raw = {}
    for v in f:
        raw[v % (1 << n)] = raw.get(v % (1 << n), 0) + 1
    return raw


def pin_regularity(o):
    """Lemma 9 (and Lemma 8 for the n-bit output), by brute force over a
    contiguous window of 2^20 (PM+32) / 2^18 (PM+64) values of one word,
    all other words and keys fixed:
      - with a_{1,r} = 1 and one level the field output is v + C mod p, so
        consecutive values step by exactly 1 mod p; the window is placed
        where v + C wraps past p, so that exactly k = p - 2^n n-bit values
        have two preimages (h and h - 2^n) and none has three;
      - with a random a_{1,r}, and with the largest admissible one, at the
        top of the word range, the field outputs are pairwise distinct and
        step by a_{1,r} mod p, and no n-bit value has more than two
        preimages;
      - with two levels (the word in the second block) the field output is
        still injective in the word."""
    rng = np.random.default_rng(18)
    for wide, W, p, amax, span in ((False, 4, P32, AMAX32, 1 << 20), (True, 8, P64, AMAX64, 1 << 18)):
        n = 8 * W
        keys = o.expand_keys64(21) if wide else o.expand_keys32(21)
        base = bytes(rng.bytes(3 * W + 2))  # four padded words, one level
        r = 1
        # a_{1,r} = 1: window across the wrap of v + C past p
        k1 = keys.copy()
        k1[r] = 1
        c0 = _sweep_word(o, wide, base, r, 0, 1, k1)[0]  # C = output at v = 0
        cross = (p - c0) % p  # first v with v + C >= p
        assert span <= cross <= (1 << n) - span, "choose another base"
        lo = cross - span // 2
        f = _sweep_word(o, wide, base, r, lo, span, k1)
        assert all((f[i + 1] - f[i]) % p == 1 for i in range(span - 1))
        assert len(set(f)) == span
        raw = _preimage_counts(f, n)
        twice = sorted(k for k, c in raw.items() if c == 2)
        assert max(raw.values()) == 2 and twice == list(range(p - (1 << n))), (wide, twice[:20])
        # random key and the largest key, at the top of the word range
        for a in (int(keys[r]), amax):
            k2 = keys.copy()
            k2[r] = a
            f = _sweep_word(o, wide, base, r, (1 << n) - span, span, k2)
            assert all((f[i + 1] - f[i]) % p == a % p for i in range(span - 1))
            assert len(set(f)) == span
            assert max(_preimage_counts(f, n).values()) <= 2
        # two levels: the swept word in the second block
        base2 = bytes(rng.bytes(128 * W + 3 * W))
        f = _sweep_word(o, wide, base2, 128 + 1, 12345, 1 << 14, keys)
        assert len(set(f)) == 1 << 14


def pin_single_key_collisions(o):
    """Almost-Delta-universality (Lemma 9, bound 3L/(p - 1 - kappa) of Sec. 5)
    on one key: two equal-length one-level messages differing in words r and
    s, every key fixed except a_{1,r} = t. Then h(x) - h(y) = t d_r + c mod p
    with d_r = x_r - y_r and c fixed, so the field outputs collide for exactly
    one t (t = -c / d_r mod p) and the n-bit outputs can collide only where
    h(x) - h(y) is 0 or +-2^n, i.e. for at most three t. The oracle is swept
    over windows of t around the three solutions the modular inverse gives
    (plus random t over the whole range): the field collision must sit
    exactly at the predicted t, n-bit collisions only at predicted values,
    and the difference must step by d_r mod p between neighbouring t."""
    rng = np.random.default_rng(19)
    for wide, W, p, amax in ((False, 4, P32, AMAX32), (True, 8, P64, AMAX64)):
        n = 8 * W
        h = (o.pm64 if wide else o.pm32)
        keys = o.expand_keys64(31) if wide else o.expand_keys32(31)
        r, s_ = 2, 0
        for _ in range(50):
            x = bytearray(rng.bytes(3 * W + 1))
            y = bytearray(x)
            y[r * W:(r + 1) * W] = rng.bytes(W)
            y[s_ * W:(s_ + 1) * W] = rng.bytes(W)
            xw, yw = _words(bytes(x), W), _words(bytes(y), W)
            d = [(a - b) % p for a, b in zip(xw, yw)]
            c = sum(int(keys[i]) * d[i] for i in range(len(d)) if i != r) % p
            inv = pow(d[r], -1, p)
            t_star = (-c * inv) % p
            cands = {t_star} | {((e - c) * inv) % p for e in (1 << n, p - (1 << n))}
            if 1 <= t_star <= amax:
                break
        else:
            raise AssertionError("no pair with an admissible colliding key")
        half = 2048
        ts = set()
        for t0 in cands:
            ts |= set(range(max(1, t0 - half), min(amax, t0 + half) + 1))
        ts |= {int.from_bytes(rng.bytes(W), "little") % amax + 1 for _ in range(2000)}
        field_hits, raw_hits = [], []
        prev = None
        for t in sorted(ts):
            k = keys.copy()
            k[r] = t
            hx = h(bytes(x), k, O.FIELD)[0]
            hy = h(bytes(y), k, O.FIELD)[0]
            diff = (hx - hy) % p
            if prev is not None and prev[0] == t - 1:
                assert (diff - prev[1]) % p == d[r], (wide, t)
            prev = (t, diff)
            if hx == hy:
                field_hits.append(t)
            if hx % (1 << n) == hy % (1 << n):
                raw_hits.append(t)
        assert field_hits == [t_star], (wide, field_hits, t_star)
        assert set(raw_hits) <= cands and t_star in raw_hits and len(raw_hits) <= 3, (wide, raw_hits)


def pin_splitmix(o):
    """Published splitmix64 outputs for state 0."""
    want = [int(x[0], 16) for x in _gold_lines("splitmix64_seed0.txt")]
    got = [int(v) for v in o.splitmix64_stream(0, len(want))]
    assert got == want, [hex(g) for g in got]


GAMMA = 0x9E3779B97F4A7C15
_SM_MUL = (0xBF58476D1CE4E5B9, 0x94D049BB133111EB)


def splitmix_seed_for(value: int, draw: int) -> int:
    """The seed whose splitmix64 stream has ``value`` as output number ``draw``
    (0-based): undo the finalizer (xorshifts and odd multipliers, inverted
    here) to get the state, then step the golden gamma back. Used to force the
    rejection path of the key expansion at a chosen draw."""
    mask = (1 << 64) - 1
    z = _inv_xorshift(value, 31, 64)
    z = _inv_xorshift((z * pow(_SM_MUL[1], -1, 1 << 64)) & mask, 27, 64)
    z = _inv_xorshift((z * pow(_SM_MUL[0], -1, 1 << 64)) & mask, 30, 64)
    return (z - (draw + 1) * GAMMA) & mask


def reject_seeds(wide: bool):
    """(seed, draw, candidate) triples whose stream puts an out-of-range a
    candidate (0 or above p - kappa - 1) or the largest admissible one at a
    chosen draw: at the first draw, in the middle of level 1, and in the
    last level."""
    if wide:
        vals = [(0, False), ((1 << 64) - 11, False), ((1 << 64) - 1, False), (AMAX64, True)]
    else:
        vals = [(0x12345678, False), (((1 << 32) - 13) << 32 | 7, False), (((1 << 32) - 1) << 32, False),
                (AMAX32 << 32 | 0xFFFFFFFF, True)]
    out = []
    for (v, ok), draw in zip(vals, (0, 77, 900, 5)):
        out.append((splitmix_seed_for(v, draw), draw, v >> (0 if wide else 32), ok))
    return out


def pin_key_expansion(o):
    """Key tables: a in [1, p - kappa - 1], drawn in storage order from the
    splitmix64 stream (PM+32 takes the top 32 bits of each output), candidates
    outside the range skipped; b are the next 8 draws, unrestricted. Seeds
    built by inverting the finalizer force a rejected candidate (or the
    largest accepted one) at a chosen draw."""
    for wide, amax, shift in ((False, AMAX32, 32), (True, AMAX64, 0)):
        forced = reject_seeds(wide)
        for seed, draw, cand, ok in forced:
            stream = [int(v) >> shift for v in o.splitmix64_stream(seed, draw + 1)]
            assert stream[draw] == cand
            k = o.expand_keys64(seed) if wide else o.expand_keys32(seed)
            if ok:
                assert int(k[draw]) == cand == amax
            else:
                assert cand not in [int(v) for v in k[:1024]]
        for seed in (0, 1, 2, 12345) + tuple(f[0] for f in forced):
            k = o.expand_keys64(seed) if wide else o.expand_keys32(seed)
            stream = [int(v) >> shift for v in o.splitmix64_stream(seed, 1100)]
            acc = [c for c in stream if 1 <= c <= amax][:1024]
            used = 0
            n_ok = 0
            while n_ok < 1024:
                if 1 <= stream[used] <= amax:
                    n_ok += 1
                used += 1
            assert [int(v) for v in k[:1024]] == acc
            assert [int(v) for v in k[1024:]] == stream[used:used + 8]
            assert all(1 <= int(v) <= amax for v in k[:1024])


def pin_key_range(o):
    """Eq. (1) keys lie in (0, p - kappa): the largest allowed key is accepted
    and the next one is rejected."""
    for wide, amax in ((False, AMAX32), (True, AMAX64)):
        _h(o, wide, b"x", _unit(wide, {(0, 3): amax}))
        if amax + 1 < (1 << (64 if wide else 32)):
            try:
                _h(o, wide, b"x", _unit(wide, {(0, 3): amax + 1}))
            except O.OracleError:
                pass
            else:
                raise AssertionError("key above range accepted")


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
