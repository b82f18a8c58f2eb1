"""Pins of the PM+128 oracle (oracle/pm128.py) against what the mathematics
fixes: the prime and its minimality, unit and all-ones keys (textbook word
extraction and checksum), a hand-expanded tree for m = 4, key ranges, and
linearity in the keys."""
from __future__ import annotations

import random

import pytest

from oracle import pm128 as O


def is_probable_prime(n: int, rounds: int = 40) -> bool:
    """Miller-Rabin with `rounds` fixed pseudo-random bases: a 'composite'
    answer is certain; a 'prime' answer errs with probability < 4^-rounds."""
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(12345)
    for _ in range(rounds):
        x = pow(rng.randrange(2, n - 1), d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_prime_and_smallest():
    assert O.P128 == 2**128 + 51
    assert is_probable_prime(O.P128)
    assert not any(is_probable_prime(2**128 + k) for k in range(1, 51))


def test_splitmix_and_key_ranges():
    g = O.splitmix64(0)
    assert next(g) == 0xE220A8397B1DCDAF  # splitmix64(0)'s first output
    a, b = O.expand_keys128(3)
    assert len(a) == 8 and all(len(r) == 128 for r in a) and len(b) == 8
    assert all(1 <= v <= 2**128 - 50 for r in a for v in r)
    assert all(0 <= v < 2**128 for v in b)
    # first key = first two draws, low half first
    g = O.splitmix64(3)
    lo, hi = next(g), next(g)
    assert a[0][0] == lo | (hi << 64)


def test_words_little_endian_and_pad():
    assert O.words(b"") == [1]
    assert O.words(bytes(range(16))) == [int.from_bytes(bytes(range(16)), "little"), 1]
    assert O.words(b"\x02\x03") == [0x010302]


def unit_keys(r):
    a = [[0] * 128 for _ in range(8)]
    a[0][r] = 1
    return a, [0] * 8


@pytest.mark.parametrize("r", [0, 5, 127])
def test_unit_key_returns_word(r):
    rng = random.Random(r)
    data = bytes(rng.randrange(256) for _ in range(16 * 127 + 3))  # one block of 128 words
    a, b = unit_keys(r)
    assert O.pm128(data, a, b, field=True) == O.words(data)[r]


def test_all_ones_is_checksum():
    rng = random.Random(7)
    data = bytes(rng.randrange(256) for _ in range(1000))
    a = [[1] * 128 for _ in range(8)]
    assert O.pm128(data, a, [0] * 8, field=True) == sum(O.words(data)) % O.P128


def test_tree_m4_by_hand():
    # m = 4, five words: level 1 makes two values, level 2 one (Fig. 1 shape)
    rng = random.Random(9)
    a = [[rng.randrange(1, 2**128 - 50) for _ in range(4)] for _ in range(8)]
    b = [rng.randrange(2**128) for _ in range(8)]
    s = [rng.randrange(2**128) for _ in range(5)]
    p = O.P128
    f10 = (b[0] + sum(a[0][i] * s[i] for i in range(4))) % p
    f11 = (b[0] + a[0][0] * s[4]) % p
    want = (b[1] + a[1][0] * f10 + a[1][1] * f11) % p
    assert O.tree(s, a, b, m=4) == want
    # one word: one level still applies (the do-while)
    assert O.tree(s[:1], a, b, m=4) == (b[0] + a[0][0] * s[0]) % p


def test_output_is_h_mod_2_128():
    a, b = O.expand_keys128(5)
    data = b"abc" * 100
    h = O.pm128(data, a, b, field=True)
    assert 0 <= h < O.P128
    assert O.pm128(data, a, b) == h % 2**128


def test_linear_in_level1_keys():
    # one level (at most 127 data words): F(a + d, b) = F(a, b) + F(d, 0) mod p
    rng = random.Random(11)
    data = bytes(rng.randrange(256) for _ in range(700))
    a, b = O.expand_keys128(6)
    d = [[rng.randrange(0, 2**127) for _ in range(128)]] + [[0] * 128] * 7
    ad = [[(x + y) for x, y in zip(a[0], d[0])]] + a[1:]
    lhs = O.pm128(data, ad, b, field=True)
    rhs = (O.pm128(data, a, b, field=True) + O.tree(O.words(data), d, [0] * 8)) % O.P128
    assert lhs == rhs
