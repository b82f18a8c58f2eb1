"""Incremental hashing (pmp_incr_*) against the oracle, bit for bit.

The digest after any sequence of appends must equal the oracle's hash of the
concatenated pieces (Sec. 4: the tree of Algorithm 1 over the words in order,
whatever the piece boundaries). Pieces are slices of one device buffer at
every byte alignment; sizes hit the block and node boundaries (128 W and
128^2 W bytes) and the level transitions up to four levels. Expected values
come from the oracle only; inputs from the seeded generators."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import gpu_util as U
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_prefixes(wide, data, cuts, keys_np, flags=0):
    """Oracle hashes of data[:c] for every c in cuts (as one ragged batch)."""
    buf = np.concatenate([data[:c] for c in cuts]) if cuts else np.zeros(0, np.uint8)
    off = np.zeros(len(cuts) + 1, np.int64)
    np.cumsum(np.asarray(cuts, np.int64), out=off[1:])
    return U.oracle_hash(W.Ragged(buf, off, wide), keys_np, flags)


def piece_sizes(wide, total, rng):
    """Piece sizes summing to `total`: boundary sizes first, then random ones."""
    Wb = 8 if wide else 4
    C = 128 * Wb
    sizes = [0, 1, 3, Wb - 1, Wb, 1, C - 7, C, C + 1, 0, 2 * C - 1, 127 * C + 5, 128 * C, 3]
    out, used = [], 0
    for s in sizes:
        if used + s > total:
            break
        out.append(s)
        used += s
    while used < total:
        s = int(min(total - used, rng.choice([1, 5, Wb + 3, C - 1, C + 9, 3 * C, 40 * C + 11, 200 * C - 3])))
        out.append(s)
        used += s
    return out


def run_pieces(wide, data, sizes, keys_np, lead, flags=0, every=True):
    """Append data in pieces of `sizes` from a device copy offset by `lead`
    bytes; digest after every piece (or only at the end). Returns (cuts,
    digests)."""
    import torch

    from paper_1609_09840_amd import pmp

    dbuf = torch.from_numpy(np.concatenate([np.zeros(lead, np.uint8), data])).to(U.dev())
    keys = U.to_dev_keys(keys_np)
    h = pmp.pmp_incr_create(wide, keys)
    outs, cuts, pos = [], [], 0
    for s in sizes:
        h.append(dbuf[lead + pos:lead + pos + s])
        pos += s
        if every:
            outs.append(h.digest(flags=flags))
            cuts.append(pos)
    if not every:
        outs.append(h.digest(flags=flags))
        cuts.append(pos)
    assert len(h) == pos
    torch.cuda.synchronize()
    got = np.concatenate([U.as_u64(o.cpu().numpy()).reshape(1, -1) for o in outs]).reshape(-1)
    h.close()
    return cuts, got


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("lead", [0, 1, 2, 3])
def test_incr_every_prefix(wide, lead):
    total = 300_000 if wide else 150_000  # three levels for both variants
    say(f"case incr prefixes: wide={wide} lead={lead} total={total}")
    rng = np.random.default_rng(700 + lead + 10 * wide)
    data = W.payload(total, 701 + lead)
    sizes = piece_sizes(wide, total, rng)
    keys_np = U.keys_for(wide, 1 + wide)
    cuts, got = run_pieces(wide, data, sizes, keys_np, lead)
    want = oracle_prefixes(wide, data, cuts, keys_np)
    assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("flags", [1, 2])
def test_incr_flags(wide, flags):
    total = 70_000
    say(f"case incr flags: wide={wide} flags={flags}")
    data = W.payload(total, 710)
    sizes = piece_sizes(wide, total, np.random.default_rng(711))
    keys_np = U.keys_for(wide, 1 + wide)
    cuts, got = run_pieces(wide, data, sizes, keys_np, 1, flags=flags)
    want = oracle_prefixes(wide, data, cuts, keys_np, flags)
    assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)


@pytest.mark.parametrize("wide", [False, True])
def test_incr_four_levels(wide):
    # more than 128^3 words: PM+32 above 8 MiB, PM+64 above 16 MiB
    total = (8 << 20) + 12345 if not wide else (16 << 20) + 777
    say(f"case incr four levels: wide={wide} total={total}")
    rng = np.random.default_rng(720 + wide)
    data = W.payload(total, 721)
    sizes = []
    used = 0
    for s in [3, (1 << 20) + 1, 5, (3 << 20) - 7, 1 << 16, 129]:
        sizes.append(s)
        used += s
    while used < total:
        s = int(min(total - used, rng.integers(1, 3 << 20)))
        sizes.append(s)
        used += s
    keys_np = U.keys_for(wide, 1 + wide)
    cuts, got = run_pieces(wide, data, sizes, keys_np, 2, every=False)
    want = oracle_prefixes(wide, data, cuts, keys_np)
    assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)


@pytest.mark.parametrize("wide", [False, True])
def test_incr_equals_batch_call(wide):
    total = 5_000_000 + 3
    say(f"case incr vs batch call: wide={wide} total={total}")
    data = W.payload(total, 730)
    keys_np = U.keys_for(wide, 1 + wide)
    sizes = [1 << 20] * 4 + [total - (4 << 20)]
    cuts, got = run_pieces(wide, data, sizes, keys_np, 0, every=False)
    rg = W.Ragged(data, np.array([0, total], np.int64), wide)
    batch = U.gpu_hash(rg, keys_np)
    want = U.oracle_hash(rg, keys_np)
    assert got[0] == batch[0] == want[0]


@pytest.mark.parametrize("wide", [False, True])
def test_incr_reset_and_digest_keeps_state(wide):
    import torch

    from paper_1609_09840_amd import pmp

    say(f"case incr reset: wide={wide}")
    data = W.payload(200_000, 740)
    keys_np = U.keys_for(wide, 1 + wide)
    keys = U.to_dev_keys(keys_np)
    dbuf = torch.from_numpy(data).to(U.dev())
    h = pmp.Incr(wide, keys)
    h.append(dbuf[:123_457])
    h.digest()  # a digest in the middle changes nothing
    h.append(dbuf[123_457:])
    d_full = h.digest()
    h.reset()
    assert len(h) == 0
    d_empty = h.digest()
    h.append(dbuf[:99_999])
    d_part = h.digest()
    torch.cuda.synchronize()
    got = np.array([U.as_u64(x.cpu().numpy())[0] for x in (d_full, d_empty, d_part)], np.uint64)
    want = oracle_prefixes(wide, data, [200_000, 0, 99_999], keys_np)
    assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
    h.close()


@pytest.mark.parametrize("wide", [False, True])
def test_incr_too_long_rejected(wide):
    import torch

    from paper_1609_09840_amd import pmp

    say(f"case incr too long: wide={wide}")
    data = W.payload(4096, 750)
    keys_np = U.keys_for(wide, 1 + wide)
    keys = U.to_dev_keys(keys_np)
    dbuf = torch.from_numpy(data).to(U.dev())
    h = pmp.Incr(wide, keys)
    h.append(dbuf[:1000])
    # rejected on the host before any launch: 2^60 bytes need more than 8 levels
    rc = pmp._lib.pmp_incr_append(h.handle, ctypes.c_void_p(dbuf.data_ptr()), 1 << 60)
    assert rc == pmp.PMP_E_TOO_LONG
    assert len(h) == 1000
    h.append(dbuf[1000:])
    d = h.digest()
    torch.cuda.synchronize()
    want = oracle_prefixes(wide, data, [4096], keys_np)
    assert U.as_u64(d.cpu().numpy())[0] == want[0]
    h.close()


@pytest.mark.parametrize("wide", [False, True])
def test_incr_full_size_string(wide):
    """A 256 MiB string (as sixteen C3 strings end to end) appended in 16 MiB
    pieces after two small ones, so that every large piece starts at an odd
    position; the workspace grows on the first large piece."""
    total = (256 << 20) + 4097
    say(f"case incr 256 MiB: wide={wide}")
    data = W.payload(total, 760)
    sizes, used = [], 0
    for s in [7, 1 << 10, (16 << 20) - 5]:
        sizes.append(s)
        used += s
    while used < total:
        s = min(total - used, 16 << 20)
        sizes.append(s)
        used += s
    keys_np = U.keys_for(wide, 1 + wide)
    cuts, got = run_pieces(wide, data, sizes, keys_np, 3, every=False)
    want = oracle_prefixes(wide, data, cuts, keys_np)
    assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
