"""PM+128 (p = 2^128 + 51) on the GPU against the oracle (oracle/pm128.py,
exact Python integers), bit for bit: edge lengths at every alignment, the
level transitions up to four levels, flags, a C2-shaped batch, tiles mixing
every length class and offsets out of order. Expected values come from the oracle only."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_util as U
from oracle import pm128 as O
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = {}


def say(*a):
    print(*a, flush=True)


def keys_for(seed):
    if seed not in KEYS:
        KEYS[seed] = O.expand_keys128(seed)
    return KEYS[seed]


def gpu128(buf, off, seed, flags=0):
    import torch

    from paper_1609_09840_amd import pmp

    a, b = keys_for(seed)
    kt = torch.from_numpy(O.key_table_u64(a, b).view(np.int64)).to(U.dev()).view(torch.uint64)
    dbuf = torch.from_numpy(buf if buf.size else np.zeros(1, np.uint8)).to(U.dev())
    if not buf.size:
        dbuf = dbuf[:0]
    doff = torch.from_numpy(off).to(U.dev())
    out = pmp.pmp_hash128(dbuf, doff, kt, flags=flags)
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.uint64)
    k = 3 if flags & 2 else 2
    o = o.reshape(-1, k)
    return [int(r[0]) | (int(r[1]) << 64) | ((int(r[2]) << 128) if k == 3 else 0) for r in o]


def oracle128(buf, off, seed, field=False):
    a, b = keys_for(seed)
    return O.batch(buf, off, a, b, field)


def check(rg_buf, rg_off, seed=1, flags=0, label=""):
    say(f"case {label}: count={len(rg_off) - 1} bytes={int(rg_off[-1] - rg_off[0])} flags={flags}")
    got = gpu128(rg_buf, rg_off, seed, flags)
    want = oracle128(rg_buf, rg_off, seed, field=bool(flags & 2))
    bad = [i for i, (g, w) in enumerate(zip(got, want)) if g != w]
    assert not bad, (label, bad[:5])


def edge_lengths():
    ls = list(range(0, 40))
    for base in (2048, 2 * 2048, 127 * 2048, 128 * 2048, 129 * 2048):
        ls += [base - 17, base - 16, base - 15, base - 1, base, base + 1, base + 16]
    return ls


@pytest.mark.parametrize("lead", [0, 1, 2, 3])
def test_pm128_edge_lengths(lead):
    rg = W.from_lengths(edge_lengths(), 900 + lead, True, lead=lead)
    check(rg.buf, rg.offsets, 1, 0, f"edge lengths lead={lead}")


@pytest.mark.parametrize("flags", [1, 2])
def test_pm128_flags(flags):
    rg = W.from_lengths([0, 5, 16, 2047, 2048, 5000, 300000], 910, True, lead=1)
    check(rg.buf, rg.offsets, 2, flags, f"flags {flags}")


def test_pm128_c2_shaped():
    rng = np.random.default_rng(920)
    rg = W.from_lengths(rng.integers(8, 257, 3000), 921, True)
    check(rg.buf, rg.offsets, 3, 0, "c2-shaped 3000")


@pytest.mark.parametrize("lead", [0, 1])
def test_pm128_tiles_mixed(lead):
    """Tiles of 64 strings mixing the one-lane lengths (up to 271 bytes), the
    longer strings of one block and strings of several blocks, with the
    boundary lengths 271 / 272 and 2031 / 2032; 700 strings (the last tile
    partial). A long string between short ones makes a tile's short strings
    span more than the stage, so both staging forms run."""
    rng = np.random.default_rng(950 + lead)
    kinds = rng.integers(0, 10, 700)
    lengths = np.where(kinds < 6, rng.integers(0, 272, 700),
                       np.where(kinds < 9, rng.integers(272, 2032, 700), rng.integers(2032, 40000, 700)))
    lengths[:8] = [271, 272, 270, 273, 2031, 2032, 0, 271]
    rg = W.from_lengths(lengths, 951 + lead, True, lead=lead)
    check(rg.buf, rg.offsets, 4, 0, f"mixed tiles lead={lead}")


def test_pm128_four_levels():
    # more than 128^3 words of 16 bytes: four levels
    n = 128**3 * 16 + 5
    rg = W.from_lengths([n, 3, 2049], 930, True, lead=3)
    check(rg.buf, rg.offsets, 1, 0, "four levels")


def test_pm128_offsets_out_of_order_hash_as_empty():
    rg = W.from_lengths([100, 50, 70], 940, True)
    off = np.array([0, 100, 40, 220, 219], np.int64)  # pairs 1 and 3 decrease
    got = gpu128(rg.buf, off, 1)
    empty = oracle128(np.zeros(0, np.uint8), np.array([0, 0], np.int64), 1)[0]
    want0 = oracle128(rg.buf, np.array([0, 100], np.int64), 1)[0]
    want2 = oracle128(rg.buf, np.array([40, 220], np.int64), 1)[0]
    assert got == [want0, empty, want2, empty]
