"""Seeded synthetic inputs for the PM+ hashing path.

This module only draws random lengths, bytes and variant choices; it holds
none of the hashing arithmetic, so the GPU library and the CPU oracle can both
be fed from it without sharing any part of the method.

Inputs mirror the paper's workloads (random byte strings, short and long; the
paper's own data came from a third-party test harness that is not used here)
and the five batch shapes this project benchmarks:

  c1  PM+32, 1024 strings x 64 B
  c2  PM+32, 2^20 strings, lengths uniform in [8, 256] B
  c3  PM+64, 64 strings x 16 MiB
  c4  2^18 strings, lengths round(LogNormal(ln 200, 2.0)) clamped to
      [1 B, 1 MiB], each string PM+32 or PM+64 with probability 1/2
  c5  serving requests: 1..4096 strings, lengths log-uniform in
      [16 B, 64 KiB], one variant per request

Payload bytes come from numpy's PCG64 generator seeded with ``data_seed``;
lengths and variant choices from a PCG64 generator seeded with ``len_seed``.
Strings are laid back to back with no alignment padding, so string starts are
arbitrary byte offsets.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KEY_SEED32 = 1
KEY_SEED64 = 2


@dataclass
class Ragged:
    """A concatenated byte buffer with CSR offsets: string i is
    ``buf[offsets[i]:offsets[i+1]]``."""

    buf: np.ndarray  # uint8
    offsets: np.ndarray  # int64, count + 1
    wide: bool  # False: PM+32, True: PM+64

    @property
    def count(self) -> int:
        return len(self.offsets) - 1

    @property
    def nbytes(self) -> int:
        return int(self.offsets[-1] - self.offsets[0])

    def string(self, i: int) -> bytes:
        return self.buf[self.offsets[i]:self.offsets[i + 1]].tobytes()


@dataclass
class Workload:
    name: str
    batches: list = field(default_factory=list)  # list[Ragged]

    @property
    def nbytes(self) -> int:
        return sum(b.nbytes for b in self.batches)

    @property
    def count(self) -> int:
        return sum(b.count for b in self.batches)


def payload(nbytes: int, data_seed: int) -> np.ndarray:
    rng = np.random.default_rng(data_seed)
    return np.frombuffer(rng.bytes(int(nbytes)), dtype=np.uint8).copy() if nbytes else np.zeros(0, np.uint8)


def from_lengths(lengths, data_seed: int, wide: bool, lead: int = 0) -> Ragged:
    """Lay strings of the given lengths back to back. ``lead`` extra bytes are
    placed before the first string (to exercise a non-zero first offset)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    offsets += lead
    buf = payload(int(offsets[-1]), data_seed)
    return Ragged(buf, offsets, wide)


def c1() -> Workload:
    return Workload("c1", [from_lengths(np.full(1024, 64), 101, False)])


def c2(count: int = 1 << 20) -> Workload:
    rng = np.random.default_rng(202)
    lengths = rng.integers(8, 257, size=count)
    return Workload("c2", [from_lengths(lengths, 102, False)])


def c3(count: int = 64, length: int = 16 << 20) -> Workload:
    return Workload("c3", [from_lengths(np.full(count, length), 103, True)])


def c4_lengths(count: int = 1 << 18, seed: int = 204):
    rng = np.random.default_rng(seed)
    raw = rng.lognormal(mean=np.log(200.0), sigma=2.0, size=count)
    lengths = np.clip(np.rint(raw), 1, 1 << 20).astype(np.int64)
    wide = rng.random(count) < 0.5
    return lengths, wide


def c4(count: int = 1 << 18) -> Workload:
    """Half PM+32, half PM+64 (per-string coin). The two variants are laid out
    in two buffers, one per batch, each in the order the strings were drawn."""
    lengths, wide = c4_lengths(count)
    b32 = from_lengths(lengths[~wide], 104, False)
    b64 = from_lengths(lengths[wide], 1104, True)
    return Workload("c4", [b32, b64])


def c5_request(rng: np.random.Generator, data_seed: int) -> Ragged:
    """One serving request: 1..4096 strings, lengths log-uniform in
    [16 B, 64 KiB], variant drawn once for the request."""
    count = int(rng.integers(1, 4097))
    lengths = np.rint(np.exp(rng.uniform(np.log(16.0), np.log(65536.0), size=count))).astype(np.int64)
    wide = bool(rng.random() < 0.5)
    return from_lengths(lengths, data_seed, wide)


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4}
