"""Hash table of variable-length keys (pmp_table_*) against the oracle.

bucket_start must equal the oracle's exactly; each bucket must hold the same
key indices as the oracle's (the order inside a bucket is unspecified), each
entry's record the key's hash, offset and length; every probe result must
equal the oracle's (smallest equal key, or -1). Expected
values come from oracle/ only; inputs from the seeded generators."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_util as U
import oracle
from oracle import table as T
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def ragged(parts):
    off = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([p.size for p in parts], out=off[1:])
    buf = np.concatenate(parts) if off[-1] else np.zeros(0, np.uint8)
    return buf, off


def key_set(n, seed, lo=0, hi=24, dup_every=5):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi, n)
    rg = W.from_lengths(lens, seed + 1, False)
    parts = [rg.buf[rg.offsets[i]:rg.offsets[i + 1]] for i in range(n)]
    if dup_every:
        for i in range(dup_every, n, dup_every):
            parts[i] = parts[int(rng.integers(0, i))]
    return parts


def queries_for(kparts, n, seed):
    """Half copies of keys (chosen at random), half fresh strings."""
    rng = np.random.default_rng(seed)
    fresh = key_set(n, seed + 7, dup_every=0)
    return [kparts[int(rng.integers(0, len(kparts)))] if q % 2 == 0 else fresh[q] for q in range(n)]


def oracle_hashes(wide, buf, off, keys_np, flags):
    return U.oracle_hash(W.Ragged(buf, off, wide), keys_np, flags)


def check_table(wide, kbuf, koff, kh, m, start, entries):
    want_start, want_entries = T.build(kh, m)
    assert np.array_equal(start, want_start)
    # same members per bucket: sorting each bucket's entries gives the oracle's
    b = T.buckets(kh, m)
    n = len(koff) - 1
    assert np.array_equal(np.sort(entries[:n]), np.arange(n))
    pos_bucket = np.searchsorted(start, np.arange(n), side="right") - 1
    assert np.array_equal(b[entries[:n]], pos_bucket)
    key = pos_bucket * (n + 1) + entries[:n]
    assert np.array_equal(entries[:n][np.argsort(key, kind="stable")], want_entries)


def entry_keys(t, koff, kh):
    """The key index of each entry, after checking the rest of its record
    (hash, offset, length) against the oracle's hashes and the offsets."""
    rec = t.entries.cpu().numpy()
    n = len(koff) - 1
    keys = rec[:n, 0]
    if n:
        assert np.array_equal(rec[:n, 1].view(np.uint64), kh[keys])
        assert np.array_equal(rec[:n, 2], koff[keys])
        assert np.array_equal(rec[:n, 3], np.diff(koff)[keys])
    return keys


def run(wide, kparts, qparts, m, flags, keys_seed):
    import torch

    from paper_1609_09840_amd import pmp

    keys_np = U.keys_for(wide, keys_seed)
    kbuf, koff = ragged(kparts)
    qbuf, qoff = ragged(qparts)
    keys = U.to_dev_keys(keys_np)
    dk, dko = U.to_dev(W.Ragged(kbuf, koff, wide))
    dq, dqo = U.to_dev(W.Ragged(qbuf, qoff, wide))
    t = pmp.pmp_table_build(wide, dk, dko, keys, m, flags)
    res = t.probe(dq, dqo)
    torch.cuda.synchronize()
    start = t.bucket_start.cpu().numpy()
    got = res.cpu().numpy()
    kh = oracle_hashes(wide, kbuf, koff, keys_np, flags)
    qh = oracle_hashes(wide, qbuf, qoff, keys_np, flags)
    assert np.array_equal(U.as_u64(t.hashes.cpu().numpy()), kh)
    entries = entry_keys(t, koff, kh)
    return kbuf, koff, kh, qbuf, qoff, qh, start, entries, got


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("m", [1, 7, 1000, 1 << 16])
def test_table_small(wide, m):
    say(f"case table small: wide={wide} m={m}")
    kparts = key_set(3000, 800 + m % 97)
    qparts = queries_for(kparts, 2000, 801)
    kbuf, koff, kh, qbuf, qoff, qh, start, entries, got = run(wide, kparts, qparts, m, 0, 1 + wide)
    check_table(wide, kbuf, koff, kh, m, start, entries)
    want_start, want_entries = T.build(kh, m)
    want = T.probe(kbuf, koff, kh, want_start, want_entries, qbuf, qoff, qh, m)
    assert U.first_mismatch(got.astype(np.uint64), want.astype(np.uint64)) is None
    assert (got >= 0).sum() >= 1000


@pytest.mark.parametrize("wide", [False, True])
def test_table_raw_outputs_and_empty_keys(wide):
    say(f"case table raw + empty: wide={wide}")
    kparts = key_set(500, 810, lo=0, hi=3)  # many empty and one-byte keys, heavy duplication
    qparts = queries_for(kparts, 300, 811) + [np.zeros(0, np.uint8)]
    m = 97
    kbuf, koff, kh, qbuf, qoff, qh, start, entries, got = run(wide, kparts, qparts, m, 1, 1 + wide)
    check_table(wide, kbuf, koff, kh, m, start, entries)
    want_start, want_entries = T.build(kh, m)
    want = T.probe(kbuf, koff, kh, want_start, want_entries, qbuf, qoff, qh, m)
    assert np.array_equal(got, want)


def test_table_c2_full():
    """C2-shaped key set (2^20 keys, 8-256 bytes, PM+32), 2^20 buckets, 2^18
    queries: the whole table against the oracle, probes on a sample."""
    import torch

    from paper_1609_09840_amd import pmp

    say("case table c2 full")
    wl = W.c2()
    rg = wl.batches[0]
    keys_np = U.keys_for(False, 1)
    m = 1 << 20
    rng = np.random.default_rng(820)
    nq = 1 << 18
    src = rng.integers(0, rg.count, nq)
    fresh = W.from_lengths(rng.integers(8, 257, nq), 821, False)
    qparts = [rg.buf[rg.offsets[j]:rg.offsets[j + 1]] if q % 2 == 0 else fresh.buf[fresh.offsets[q]:fresh.offsets[q + 1]]
              for q, j in enumerate(src)]
    qbuf, qoff = ragged(qparts)
    keys = U.to_dev_keys(keys_np)
    dk, dko = U.to_dev(rg)
    dq, dqo = U.to_dev(W.Ragged(qbuf, qoff, False))
    t = pmp.pmp_table_build(False, dk, dko, keys, m)
    res = t.probe(dq, dqo)
    torch.cuda.synchronize()
    kh = U.oracle_hash(rg, keys_np)
    assert np.array_equal(U.as_u64(t.hashes.cpu().numpy()), kh)
    check_table(False, rg.buf, rg.offsets, kh, m, t.bucket_start.cpu().numpy(), entry_keys(t, rg.offsets, kh))
    got = res.cpu().numpy()
    qh = U.oracle_hash(W.Ragged(qbuf, qoff, False), keys_np)
    want_start, want_entries = T.build(kh, m)
    sample = np.concatenate([np.arange(64), rng.choice(nq, 3000, replace=False), np.arange(nq - 64, nq)])
    want = T.probe(rg.buf, rg.offsets, kh, want_start, want_entries, qbuf, qoff, qh, m, which=sample)
    assert np.array_equal(got[sample], want)
    # every hit is a key with the query's hash and length (all queries)
    hit = got >= 0
    assert np.array_equal(kh[got[hit]], qh[hit])
    klen = np.diff(rg.offsets)
    assert np.array_equal(klen[got[hit]], np.diff(qoff)[hit])
    assert hit.sum() >= nq // 2


def test_table_no_keys():
    import torch

    from paper_1609_09840_amd import pmp

    say("case table with no keys")
    keys = U.to_dev_keys(U.keys_for(False, 1))
    dk = torch.zeros(1, dtype=torch.uint8, device=U.dev())[:0]
    dko = torch.zeros(1, dtype=torch.int64, device=U.dev())
    t = pmp.pmp_table_build(False, dk, dko, keys, 16)
    qbuf, qoff = ragged(key_set(10, 830))
    dq, dqo = U.to_dev(W.Ragged(qbuf, qoff, False))
    res = t.probe(dq, dqo)
    torch.cuda.synchronize()
    assert np.array_equal(t.bucket_start.cpu().numpy(), np.zeros(17, np.int64))
    assert (res.cpu().numpy() == -1).all()


@pytest.mark.parametrize("wide", [False, True])
def test_table_all_hashes_equal(wide):
    """Level-1 keys all zero: every key (one block each) hashes to b_1, so
    every probe meets keys of equal hash and length whose bytes differ (the
    probe's compare-every-candidate path)."""
    import torch

    from paper_1609_09840_amd import pmp

    say(f"case table all hashes equal: wide={wide}")
    keys_np = U.keys_for(wide, 1 + wide).copy()
    keys_np[:8 * 128] = 0  # every a = 0 (allowed: zero keys cannot overflow); b kept
    kparts = key_set(400, 850, lo=4, hi=12, dup_every=3)
    qparts = queries_for(kparts, 300, 851)
    kbuf, koff = ragged(kparts)
    qbuf, qoff = ragged(qparts)
    keys = U.to_dev_keys(keys_np)
    dk, dko = U.to_dev(W.Ragged(kbuf, koff, wide))
    dq, dqo = U.to_dev(W.Ragged(qbuf, qoff, wide))
    m = 64
    t = pmp.pmp_table_build(wide, dk, dko, keys, m)
    res = t.probe(dq, dqo)
    torch.cuda.synchronize()
    kh = oracle_hashes(wide, kbuf, koff, keys_np, 0)
    qh = oracle_hashes(wide, qbuf, qoff, keys_np, 0)
    assert len(set(kh.tolist())) == 1  # one hash for all keys
    check_table(wide, kbuf, koff, kh, m, t.bucket_start.cpu().numpy(), entry_keys(t, koff, kh))
    want_start, want_entries = T.build(kh, m)
    want = T.probe(kbuf, koff, kh, want_start, want_entries, qbuf, qoff, qh, m)
    got = res.cpu().numpy()
    assert np.array_equal(got, want)
    assert (got >= 0).sum() >= 140


@pytest.mark.parametrize("wide", [False, True])
def test_table_all_hashes_equal_long(wide):
    """As above with keys of 1 to 300 bytes (one block each), so that equal
    hash and length leave the bytes to decide: the queries copy keys whole
    or with one byte changed at the first, the last or a position next to a
    16-byte granule or 64-byte compare-round boundary (bytes 0, 15, 16, 63,
    64, 127, 128, 191, 192, 255 and the last), and lie at every offset mod 16
    from the keys."""
    import torch

    from paper_1609_09840_amd import pmp

    say(f"case table all hashes equal, long keys: wide={wide}")
    keys_np = U.keys_for(wide, 3 + wide).copy()
    keys_np[:8 * 128] = 0
    rng = np.random.default_rng(870)
    kparts = key_set(600, 871, lo=1, hi=301, dup_every=7)
    qparts = []
    for q in range(900):
        src = kparts[int(rng.integers(0, len(kparts)))].copy()
        if q % 3 == 1:
            cands = [p for p in (0, 15, 16, 63, 64, 127, 128, 191, 192, 255, src.size - 1) if p < src.size]
            p = cands[int(rng.integers(0, len(cands)))]
            src[p] ^= np.uint8(1 + rng.integers(0, 255))
        elif q % 3 == 2:
            src = rng.integers(0, 256, src.size).astype(np.uint8)
        # a filler of 0..15 bytes moves the next query's offset mod 16
        qparts.append(src)
        qparts.append(rng.integers(0, 256, int(rng.integers(0, 16))).astype(np.uint8))
    kbuf, koff = ragged(kparts)
    qbuf, qoff = ragged(qparts)
    keys = U.to_dev_keys(keys_np)
    dk, dko = U.to_dev(W.Ragged(kbuf, koff, wide))
    dq, dqo = U.to_dev(W.Ragged(qbuf, qoff, wide))
    m = 64
    t = pmp.pmp_table_build(wide, dk, dko, keys, m)
    res = t.probe(dq, dqo)
    torch.cuda.synchronize()
    kh = oracle_hashes(wide, kbuf, koff, keys_np, 0)
    qh = oracle_hashes(wide, qbuf, qoff, keys_np, 0)
    assert len(set(kh.tolist())) == 1
    want_start, want_entries = T.build(kh, m)
    want = T.probe(kbuf, koff, kh, want_start, want_entries, qbuf, qoff, qh, m)
    got = res.cpu().numpy()
    assert np.array_equal(got, want)
    assert (got[0::6] >= 0).all()  # the whole copies
    assert (got[2::6] < 0).sum() >= 100  # most one-byte changes find no key
