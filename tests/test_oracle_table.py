"""Pins of the hash-table oracle (oracle/table.py) against what the definition
fixes independently of it: brute-force search over every key, explicit bucket
membership, and the single-bucket special case. Inputs are seeded; hashes
come from the PM+ oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import table as T
from paper_1609_09840_amd import workloads as W


def key_set(n, seed, dup_every=5):
    """n short keys with deliberate duplicates (every dup_every-th key repeats
    an earlier one) and a few empty keys."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 24, n)
    lens[::17] = 0
    rg = W.from_lengths(lens, seed + 1, False)
    parts = [rg.buf[rg.offsets[i]:rg.offsets[i + 1]] for i in range(n)]
    for i in range(dup_every, n, dup_every):
        parts[i] = parts[int(rng.integers(0, i))]
    off = np.zeros(n + 1, np.int64)
    np.cumsum([p.size for p in parts], out=off[1:])
    buf = np.concatenate(parts) if off[-1] else np.zeros(0, np.uint8)
    return buf, off


def hashes(buf, off, wide=False):
    keys = oracle.load().expand_keys64(2) if wide else oracle.load().expand_keys32(1)
    return oracle.load().batch(wide, buf, off, keys, oracle.MIXED).reshape(-1).astype(np.uint64)


@pytest.mark.parametrize("m", [1, 7, 64, 1000])
def test_build_membership(m):
    buf, off = key_set(300, 11)
    h = hashes(buf, off)
    start, entries = T.build(h, m)
    assert start[0] == 0 and start[-1] == len(off) - 1
    for b in range(m):
        members = [i for i in range(len(off) - 1) if int(h[i]) % m == b]
        assert list(entries[start[b]:start[b + 1]]) == members  # increasing key order


def test_single_bucket_is_identity():
    buf, off = key_set(50, 12)
    start, entries = T.build(hashes(buf, off), 1)
    assert list(start) == [0, 50] and list(entries) == list(range(50))


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("m", [1, 13, 256])
def test_probe_is_first_equal_key(wide, m):
    buf, off = key_set(400, 13 + wide)
    kh = hashes(buf, off, wide)
    qbuf, qoff = key_set(200, 14 + wide, dup_every=3)
    # half the queries copy keys, the rest are fresh strings
    parts = [qbuf[qoff[i]:qoff[i + 1]] if i % 2 else buf[off[(3 * i) % 400]:off[(3 * i) % 400 + 1]]
             for i in range(200)]
    qoff = np.zeros(201, np.int64)
    np.cumsum([p.size for p in parts], out=qoff[1:])
    qbuf = np.concatenate(parts)
    qh = hashes(qbuf, qoff, wide)
    start, entries = T.build(kh, m)
    got = T.probe(buf, off, kh, start, entries, qbuf, qoff, qh, m)
    keys = [buf[off[i]:off[i + 1]].tobytes() for i in range(400)]
    want = [next((i for i, k in enumerate(keys) if k == parts[q].tobytes()), -1) for q in range(200)]
    assert list(got) == want
    assert (got >= 0).sum() >= 100  # the copied keys are found
    # the pin tells the first equal key from a later one: some queries match
    # several keys, and a probe that returned the last match would fail
    last = [max((i for i, k in enumerate(keys) if k == parts[q].tobytes()), default=-1) for q in range(200)]
    assert last != want
