"""Test oracle for the hash-table use of PM+ (Sec. 1 and Sec. 3: a hash family
picks the bucket of a key; Lemma 1 and Lemma 8: h mod M keeps the family
almost universal and regular).

THIS IS TEST INFRASTRUCTURE. Only the test suite may import it. The GPU library
never imports, links or calls anything here, and nothing here imports the
library.

Plain definitions, written out:
  bucket(i)        = h_i mod M, with h_i the n-bit output of key i;
  table            = for each bucket b, the key indices i with bucket(i) = b
                     (bucket_start[b] .. bucket_start[b + 1] in a CSR layout);
  probe(query q)   = the smallest key index i whose bytes equal q's bytes, or
                     -1 if there is none (equal bytes give equal hashes, so
                     only q's bucket needs to be searched).
"""
from __future__ import annotations

import numpy as np


def buckets(hashes: np.ndarray, m: int) -> np.ndarray:
    """bucket(i) = h_i mod M."""
    return (hashes.astype(np.uint64) % np.uint64(m)).astype(np.int64)


def build(hashes: np.ndarray, m: int) -> tuple[np.ndarray, np.ndarray]:
    """(bucket_start[M + 1], entries[n]): entries grouped by bucket, each
    bucket's entries in increasing key order (a stable sort by bucket)."""
    b = buckets(hashes, m)
    counts = np.bincount(b, minlength=m).astype(np.int64)
    start = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=start[1:])
    entries = np.argsort(b, kind="stable").astype(np.int64)
    return start, entries


def key_bytes(buf: np.ndarray, offsets: np.ndarray, i: int) -> bytes:
    return buf[offsets[i]:offsets[i + 1]].tobytes()


def probe(kbuf, koffsets, khashes, start, entries, qbuf, qoffsets, qhashes, m: int, which=None) -> np.ndarray:
    """Probe results for the queries `which` (default: all), one by one."""
    idx = range(len(qoffsets) - 1) if which is None else which
    out = []
    for q in idx:
        qb = key_bytes(qbuf, qoffsets, q)
        b = int(np.uint64(qhashes[q]) % np.uint64(m))
        best = -1
        for e in range(int(start[b]), int(start[b + 1])):
            i = int(entries[e])
            if key_bytes(kbuf, koffsets, i) == qb and (best < 0 or i < best):
                best = i
        out.append(best)
    return np.asarray(out, np.int64)
