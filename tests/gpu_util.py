"""Helpers shared by the GPU tests: move a Ragged batch to the device, run the
library, run the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle

MODES = {0: oracle.MIXED, 1: oracle.RAW, 2: oracle.FIELD}  # library flags -> oracle modes


def dev():
    import torch

    return torch.device("cuda:0")


def keys_for(wide: bool, seed: int):
    """Key table for seed, from the oracle's own expansion: no expected value
    of a GPU test depends on a library output (the library's expansion is
    compared with this one in test_keys.py)."""
    o = oracle.load()
    return o.expand_keys64(seed) if wide else o.expand_keys32(seed)


def to_dev_keys(keys_np: np.ndarray):
    import torch

    wide = keys_np.dtype == np.uint64
    t = torch.from_numpy(keys_np.view(np.int64) if wide else keys_np.view(np.int32)).to(dev())
    return t.view(torch.uint64 if wide else torch.uint32)


def to_dev(rg):
    import torch

    buf = torch.from_numpy(rg.buf if rg.buf.size else np.zeros(1, np.uint8)).to(dev())
    if not rg.buf.size:
        buf = buf[:0]
    off = torch.from_numpy(rg.offsets).to(dev())
    return buf, off


def gpu_hash(rg, keys_np, flags=0, plan=None, buf=None, off=None):
    import torch

    from paper_1609_09840_amd import pmp

    if buf is None:
        buf, off = to_dev(rg)
    keys = to_dev_keys(keys_np)
    f = pmp.pmp_hash64 if rg.wide else pmp.pmp_hash32
    out = f(buf, off, keys, flags=flags, plan=plan)
    torch.cuda.synchronize()
    return as_u64(out.cpu().numpy())


def as_u64(a: np.ndarray) -> np.ndarray:
    return a.reshape(-1).astype(np.uint64)


def oracle_hash(rg, keys_np, flags=0, nthreads=8):
    return as_u64(oracle.load().batch(rg.wide, rg.buf, rg.offsets, keys_np, MODES[flags], nthreads=nthreads))


def first_mismatch(got, want):
    bad = np.nonzero(got != want)[0]
    return None if bad.size == 0 else (int(bad[0]), int(got[bad[0]]), int(want[bad[0]]), int(bad.size))


def sample_ragged(rg, idx):
    """The strings idx of rg (in that order) as a Ragged of their own, for the
    oracle to hash one by one."""
    from paper_1609_09840_amd import workloads as W

    idx = np.asarray(idx, dtype=np.int64)
    lens = rg.offsets[idx + 1] - rg.offsets[idx]
    off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    parts = [rg.buf[rg.offsets[i]:rg.offsets[i + 1]] for i in idx]
    buf = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return W.Ragged(buf, off, rg.wide)
