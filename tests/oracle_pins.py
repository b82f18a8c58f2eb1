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
                            output is a bijection of the swept word; the n-bit
                            output has at most 2 preimages (Lemma 8).
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


def pin_regularity(o):
    """Lemma 9 / Lemma 8, brute force over a swept word: with all other words
    and all keys fixed, distinct values of word r give distinct field
    outputs (an injective affine map), and n-bit outputs have at most two
    preimages."""
    rng = np.random.default_rng(18)
    for wide, W in ((False, 4), (True, 8)):
        keys = o.expand_keys64(21) if wide else o.expand_keys32(21)
        base = bytearray(rng.bytes(3 * W + 2))
        seen_f, seen_r = set(), {}
        vals = [int(v) for v in rng.choice(1 << 16, size=1500, replace=False)]
        vals += [(1 << 8 * W) - 1 - v for v in range(40)]
        for v in vals:
            base[W:2 * W] = v.to_bytes(W, "little")
            f = _h(o, wide, bytes(base), keys)[0]
            assert f not in seen_f
            seen_f.add(f)
            r = f % (1 << 8 * W)
            seen_r[r] = seen_r.get(r, 0) + 1
            assert seen_r[r] <= 2


def pin_collision_bound(o):
    """Almost-Delta-universality (Lemma 9, final bound 3L/(p-1-kappa)): over
    random key tables, pairs of tiny distinct messages collide in their n-bit
    output no more often than the bound allows (expected count far below 1)."""
    msgs = [b"", b"\x00", b"\x01", b"\x00\x00\x00\x00", b"\x01\x00\x00\x00", b"a", b"b"]
    draws = 300
    for wide, p, kappa in ((False, P32, 28), (True, P64, 24)):
        coll = 0
        for s in range(draws):
            keys = o.expand_keys64(1000 + s) if wide else o.expand_keys32(1000 + s)
            outs = [_h(o, wide, m, keys, O.RAW)[0] for m in msgs]
            coll += len(outs) - len(set(outs))
        pairs = draws * len(msgs) * (len(msgs) - 1) // 2
        bound = 3 * 1 / (p - 1 - kappa) * pairs
        assert coll <= bound + 3 * (bound ** 0.5) + 1e-9, (wide, coll, bound)


def pin_splitmix(o):
    """Published splitmix64 outputs for state 0."""
    want = [int(x[0], 16) for x in _gold_lines("splitmix64_seed0.txt")]
    got = [int(v) for v in o.splitmix64_stream(0, len(want))]
    assert got == want, [hex(g) for g in got]


def pin_key_expansion(o):
    """Key tables: a in [1, p - kappa - 1], drawn in storage order from the
    splitmix64 stream (PM+32 takes the top 32 bits of each output), candidates
    outside the range skipped; b are the next 8 draws, unrestricted."""
    for wide, amax, shift in ((False, AMAX32, 32), (True, AMAX64, 0)):
        for seed in (0, 1, 2, 12345):
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
