"""GPU path vs the CPU oracle, bit for bit, through the C ABI.

Every case prints what it runs before touching the GPU. Inputs are the
seeded generators of paper_1609_09840_amd.workloads; expected values come
from the oracle only."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_util as U
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def check(rg, keys_np, flags=0, label=""):
    say(f"case {label}: wide={rg.wide} count={rg.count} bytes={rg.nbytes} flags={flags}")
    got = U.gpu_hash(rg, keys_np, flags)
    want = U.oracle_hash(rg, keys_np, flags)
    assert got.shape == want.shape
    assert U.first_mismatch(got, want) is None, (label, U.first_mismatch(got, want))


def edge_lengths(wide):
    Wb = 8 if wide else 4
    blk = 128 * Wb
    ls = list(range(0, 3 * Wb + 2))
    for base in (blk, 2 * blk, 64 * blk, 127 * blk, 128 * blk, 129 * blk, 128 * 128 * blk // 128 * 2):
        ls += [base - Wb - 1, base - Wb, base - 1, base, base + 1, base + Wb]
    return [x for x in ls if x >= 0]


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("lead", [0, 1, 2, 3])
def test_edge_lengths(wide, lead):
    """Word, block and node boundaries, every start alignment."""
    rg = W.from_lengths(edge_lengths(wide), 300 + lead, wide, lead=lead)
    check(rg, U.keys_for(wide, 11), 0, f"edges lead={lead}")


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("flags", [0, 1, 2])
def test_output_modes(wide, flags):
    rng = np.random.default_rng(21)
    lengths = np.concatenate([[0, 1, 7, 8, 9], rng.integers(0, 5000, size=500)])
    rg = W.from_lengths(lengths, 22, wide, lead=5)
    check(rg, U.keys_for(wide, 23), flags, "modes")


@pytest.mark.parametrize("wide", [False, True])
def test_three_and_four_levels(wide):
    """Strings that need 3 and 4 tree levels, cut at node boundaries."""
    Wb = 8 if wide else 4
    node = 128 * 128 * Wb  # bytes of one level-2 node
    lengths = [node - Wb, node, node + 1, 3 * node + 17, 128 * node - Wb, 128 * node, 128 * node + 5]
    rg = W.from_lengths(lengths, 31, wide, lead=3)
    check(rg, U.keys_for(wide, 32), 2, "levels")


@pytest.mark.parametrize("wide", [False, True])
def test_max_keys_max_data(wide):
    """Largest admissible keys and all-0xff data: the largest block sums."""
    from paper_1609_09840_amd import pmp

    keys = U.keys_for(wide, 1)
    amax = (1 << 64) - 12 if wide else (1 << 32) - 14
    keys[:1024] = amax
    keys[1024:] = (1 << 64) - 1 if wide else (1 << 32) - 1
    assert (pmp.pmp_check_keys64 if wide else pmp.pmp_check_keys32)(keys) == 0
    lengths = [0, 1, 500, 1016, 1024, 5000, 70000, 300000]
    rg = W.from_lengths(lengths, 41, wide)
    rg.buf[:] = 0xFF
    for flags in (0, 2):
        check(rg, keys, flags, "max")


@pytest.mark.parametrize("wide", [False, True])
def test_zero_keys(wide):
    """All-zero keys (accepted) give b_1 for one block and the tree of b's."""
    keys = np.zeros(1032, dtype=np.uint64 if wide else np.uint32)
    keys[1024:] = np.arange(1, 9)
    rg = W.from_lengths([0, 5, 600, 2000, 200000], 42, wide)
    check(rg, keys, 2, "zero keys")


def test_c1_full():
    wl = W.c1()
    check(wl.batches[0], U.keys_for(False, W.KEY_SEED32), 0, "c1")


def test_c2_slice():
    wl = W.c2(count=1 << 14)
    check(wl.batches[0], U.keys_for(False, W.KEY_SEED32), 0, "c2 2^14")


def test_c3_small():
    wl = W.c3(count=3, length=(16 << 20) // 8 + 1000)
    check(wl.batches[0], U.keys_for(True, W.KEY_SEED64), 0, "c3 small")


def test_c4_slice_mixed_launch():
    """Both variants in ONE launch (pmp_hash_mixed) vs the oracle."""
    import torch

    from paper_1609_09840_amd import pmp

    wl = W.c4(count=1 << 13)
    outs, wants = [], []
    batches = []
    keep = []
    for rg in wl.batches:
        kn = U.keys_for(rg.wide, W.KEY_SEED64 if rg.wide else W.KEY_SEED32)
        buf, off = U.to_dev(rg)
        keys = U.to_dev_keys(kn)
        out = torch.empty(rg.count, dtype=torch.uint64 if rg.wide else torch.uint32, device=U.dev())
        keep += [buf, off, keys, out]
        batches.append(pmp.make_batch(rg.wide, buf, off, keys, out))
        outs.append(out)
        wants.append(U.oracle_hash(rg, kn))
    say(f"case c4 mixed: {wl.count} strings, {wl.nbytes} bytes")
    pmp.pmp_hash_mixed(batches[0], batches[1])
    torch.cuda.synchronize()
    for out, want in zip(outs, wants):
        got = U.as_u64(out.cpu().numpy())
        assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
    assert pmp.pmp_plan_status() == 0


def test_alone_equals_in_batch():
    """A string hashes the same alone as inside any batch (batch invariance)."""
    rng = np.random.default_rng(51)
    for wide in (False, True):
        lengths = rng.integers(0, 200000, size=40)
        rg = W.from_lengths(lengths, 52, wide, lead=2)
        keys = U.keys_for(wide, 53)
        full = U.gpu_hash(rg, keys, 2)
        for i in (0, 7, 39):
            one = W.Ragged(rg.buf, rg.offsets[i:i + 2].copy(), wide)
            got = U.gpu_hash(one, keys, 2)
            stride = 2 if wide else 1
            assert np.array_equal(got, full[stride * i:stride * (i + 1)])


def test_empty_and_zero_count():
    import torch

    from paper_1609_09840_amd import pmp

    rg = W.from_lengths([0, 0, 0], 61, False)
    check(rg, U.keys_for(False, 62), 0, "empties")
    buf = torch.zeros(4, dtype=torch.uint8, device=U.dev())
    off = torch.zeros(1, dtype=torch.int64, device=U.dev())
    keys = U.to_dev_keys(U.keys_for(False, 62))
    out = pmp.pmp_hash32(buf, off, keys)
    torch.cuda.synchronize()
    assert out.numel() == 0


def test_misaligned_buffer_pointer():
    """The buffer pointer itself unaligned (a view one byte in)."""
    import torch

    from paper_1609_09840_amd import pmp

    for wide in (False, True):
        rg = W.from_lengths([5, 100, 1000, 70000, 3], 71, wide)
        raw = torch.from_numpy(np.concatenate([[0xAB], rg.buf, [0xCD]]).astype(np.uint8)).to(U.dev())
        buf = raw[1:1 + rg.buf.size]
        off = torch.from_numpy(rg.offsets).to(U.dev())
        keys_np = U.keys_for(wide, 72)
        out = (pmp.pmp_hash64 if wide else pmp.pmp_hash32)(buf, off, U.to_dev_keys(keys_np), flags=2,
                                                           buf_bytes=rg.buf.size)
        torch.cuda.synchronize()
        got = U.as_u64(out.cpu().numpy())
        assert U.first_mismatch(got, U.oracle_hash(rg, keys_np, 2)) is None


def test_bad_offsets_reported():
    """Decreasing offsets: status PMP_E_OFFSETS, the good strings still hash."""
    import torch

    from paper_1609_09840_amd import pmp

    plan = pmp.Plan(0)
    rg = W.from_lengths([10, 20, 30, 40], 81, False)
    offs = rg.offsets.copy()
    offs[2] = offs[1] - 5  # string 1 runs backwards
    buf = torch.from_numpy(rg.buf).to(U.dev())
    off = torch.from_numpy(offs).to(U.dev())
    keys_np = U.keys_for(False, 82)
    out = pmp.pmp_hash32(buf, off, U.to_dev_keys(keys_np), flags=2, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_E_OFFSETS
    assert plan.status() == pmp.PMP_OK  # cleared
    got = U.as_u64(out.cpu().numpy())
    want = U.oracle_hash(W.Ragged(rg.buf, np.array([offs[0], offs[1]]), False), keys_np, 2)
    assert got[0] == want[0]
    plan.close()


@pytest.mark.parametrize("wide", [False, True])
def test_bad_offsets_string_before_the_first(wide):
    """A string that runs backwards lets the next string start in front of
    the first one of its tile, with short strings after it. With the whole
    batch in one wave's share, every string with valid offsets still hashes
    (the one-lane strings of the tile are then copied chunk by chunk, in
    passes that stop at the first string that does not fit)."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(87)
    buf = rng.integers(0, 256, size=4096, dtype=np.uint8)
    offs = np.array([200, 300, 0, 250, 260, 270, 280, 290, 300] + list(range(310, 3000, 37)), dtype=np.int64)
    say(f"case bad-offsets-in-front: wide={wide} count={len(offs) - 1}")
    plan = pmp.Plan(0)
    plan.tune(0, 0, 1 << 26, 1)  # one wave: its share is the whole batch
    keys_np = U.keys_for(wide, 88)
    fn = pmp.pmp_hash64 if wide else pmp.pmp_hash32
    out = fn(torch.from_numpy(buf).to(U.dev()), torch.from_numpy(offs).to(U.dev()), U.to_dev_keys(keys_np), flags=0,
             plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_E_OFFSETS
    got = U.as_u64(out.cpu().numpy())  # one output word per string
    for k in range(len(offs) - 1):
        if offs[k] > offs[k + 1]:
            continue
        want = U.oracle_hash(W.Ragged(buf, offs[k:k + 2].copy(), wide), keys_np, 0)
        assert got[k] == want[0], k
    plan.close()


TILE_PAIRS = [(8, 16), (8, 8), (16, 16), (4, 16), (16, 8), (4, 8)]


def test_tiles_agree():
    """Every compiled lanes-per-block pair gives the same results."""
    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(91)
    for wide in (False, True):
        rg = W.from_lengths(rng.integers(0, 300000, size=30), 92, wide, lead=1)
        keys = U.keys_for(wide, 93)
        want = U.oracle_hash(rg, keys, 2)
        for g32, g64 in TILE_PAIRS:
            plan = pmp.Plan(0)
            plan.set_tile(False, g32)
            plan.set_tile(True, g64)
            say(f"case tiles ({g32}, {g64}) wide={wide}")
            got = U.gpu_hash(rg, keys, 2, plan=plan)
            assert U.first_mismatch(got, want) is None, (g32, g64, U.first_mismatch(got, want))
            plan.close()


@pytest.mark.parametrize("wide", [False, True])
def test_last_block_ends(wide):
    """Strings of 2 to 33 blocks (the medium path up to 32, then a long one)
    whose last block holds r bytes, r next to every 16-byte piece boundary
    that a lane of a group of 4, 8 or 16 lanes can own, at all four
    alignments, for every compiled tile pair: the pieces of a last block
    past the string's end are read from elsewhere and must not count."""
    from paper_1609_09840_amd import pmp

    bw = 128 * (8 if wide else 4)  # bytes per block
    rs = sorted({r for p in range(0, bw, 16) for r in (p - 1, p, p + 1) if 0 <= r < bw} | {bw - 1})
    rng = np.random.default_rng(131 + wide)
    blocks = rng.integers(1, 33, size=len(rs))  # full blocks before the last one
    lengths = np.array([int(b) * bw + r for b, r in zip(blocks, rs)], dtype=np.int64)
    keys = U.keys_for(wide, 133)
    for lead in range(4):
        rg = W.from_lengths(lengths, 134 + lead, wide, lead=lead)
        want = U.oracle_hash(rg, keys, 2)
        for g32, g64 in TILE_PAIRS:
            plan = pmp.Plan(0)
            plan.set_tile(False, g32)
            plan.set_tile(True, g64)
            say(f"case last-block ends wide={wide} lead={lead} tiles ({g32}, {g64}) count={rg.count}")
            got = U.gpu_hash(rg, keys, 2, plan=plan)
            assert U.first_mismatch(got, want) is None, (lead, g32, g64, U.first_mismatch(got, want))
            plan.close()


@pytest.mark.parametrize("shares", [1, 4])
def test_split_by_count(shares):
    """Shares cut by string count (PMP_ALPHA_BY_COUNT, no offset search):
    every string whole in one wave's share, long ones with several level-2
    nodes included; one batch per variant, then five batches in one launch."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(97 + shares)
    specs = []
    for k, wide in enumerate((False, True, False, True, False)):
        lengths = np.concatenate([rng.integers(0, 272, 500), rng.integers(272, 40000, 60), [0, 300000, 1, 200000]])
        rng.shuffle(lengths)
        specs.append(W.from_lengths(lengths[: 300 + 100 * k], 98 + k, wide, lead=k))
    plan = pmp.Plan(0)
    plan.tune(0, pmp.PMP_ALPHA_BY_COUNT, 0, shares)
    for rg in specs[:2]:
        keys = U.keys_for(rg.wide, 99)
        say(f"case by-count shares={shares} wide={rg.wide} count={rg.count}")
        got = U.gpu_hash(rg, keys, 2, plan=plan)
        want = U.oracle_hash(rg, keys, 2)
        assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
    say(f"case by-count shares={shares} five batches")
    k32, k64 = U.keys_for(False, 99), U.keys_for(True, 99)
    d32, d64 = U.to_dev_keys(k32), U.to_dev_keys(k64)
    keep, batches = [], []
    for rg in specs:
        buf, off = U.to_dev(rg)
        out = torch.zeros(rg.count, dtype=torch.uint64 if rg.wide else torch.uint32, device=U.dev())
        keep.append((rg, out, buf, off))
        batches.append(pmp.make_batch(rg.wide, buf, off, d64 if rg.wide else d32, out, 0))
    pmp.pmp_hash_many(batches, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_OK
    for rg, out, _, _ in keep:
        got = U.as_u64(out.cpu().numpy())
        want = U.oracle_hash(rg, k64 if rg.wide else k32, 0)
        assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
    plan.close()


def test_plain_form_matches():
    """The one-string-per-launch baseline gives identical results."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(95)
    for wide in (False, True):
        rg = W.from_lengths(np.concatenate([[0, 1, 511, 512, 1024], rng.integers(0, 100000, size=20)]), 96, wide)
        keys_np = U.keys_for(wide, 97)
        buf, _ = U.to_dev(rg)
        keys = U.to_dev_keys(keys_np)
        for flags in (0, 2):
            out = torch.empty(rg.count * (2 if (wide and flags == 2) else 1),
                              dtype=torch.uint64 if (wide or flags == 2) else torch.uint32, device=U.dev())
            scratch = torch.empty(1 << 20, dtype=torch.uint8, device=U.dev())
            pmp.pmp_hash_plain(wide, buf, rg.offsets, keys, out, flags, scratch)
            torch.cuda.synchronize()
            got = U.as_u64(out.cpu().numpy())
            assert U.first_mismatch(got, U.oracle_hash(rg, keys_np, flags)) is None


# --- field reduction (Sec. 6.2 fold + Algorithm 2) vs exact integers --------
def _fold_cases(n, k, rng, count):
    M = (1 << n) - 1
    w0s = [0, 1, k - 1, k, 2 * k - 1, 2 * k, M - k * k, M - 2 * k, M - k, M - 1, M]
    w1s = [0, 1, 2, M // k, M // k + 1, M - 1, M]
    w2s = [0, 1, 2, 64, 127, 128]
    cases = [(a, b, c) for a in w0s for b in w1s for c in w2s]
    # sums S = b + sum a_i s_i of max keys and max data
    amax = (1 << n) - k + 1
    for t in range(1, 129):
        S = (1 << n) - 1 + t * amax * M
        cases.append((S & M, (S >> n) & M, S >> (2 * n)))
    for _ in range(count):
        S = int.from_bytes(rng.bytes(2 * n // 8 + 1), "little") % (129 << (2 * n))
        cases.append((S & M, (S >> n) & M, S >> (2 * n)))
    return cases


@pytest.mark.parametrize("wide", [False, True])
def test_fold_matches_exact_mod(wide):
    import torch

    from paper_1609_09840_amd import pmp

    n, k = (64, 13) if wide else (32, 15)
    p = (1 << n) + k
    rng = np.random.default_rng(7)
    cases = _fold_cases(n, k, rng, 100000)
    say(f"case fold wide={wide}: {len(cases)} sums")
    w0 = np.array([c[0] for c in cases], dtype=np.uint64 if wide else np.uint32)
    w1 = np.array([c[1] for c in cases], dtype=np.uint64 if wide else np.uint32)
    w2 = np.array([c[2] for c in cases], dtype=np.uint32)
    tdev = lambda a: torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a.view(np.int32)).to(U.dev())
    z = torch.zeros(len(cases) * (2 if wide else 1), dtype=torch.int64, device=U.dev())
    pmp.pmp_debug_fold(wide, tdev(w0), tdev(w1), tdev(w2), z)
    torch.cuda.synchronize()
    zz = z.cpu().numpy().view(np.uint64)
    for idx, (a, b, c) in enumerate(cases):
        S = a + (b << n) + (c << (2 * n))
        got = (int(zz[2 * idx]) + (int(zz[2 * idx + 1]) << 64)) if wide else int(zz[idx])
        assert got == S % p, (a, b, c, got, S % p)


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("lead", [0, 3])
def test_stage_overflow_passes(wide, lead):
    """Runs of the longest one-lane strings (their chunks overflow the LDS
    stage, so a tile takes several passes) and of the longest medium strings
    (their block tasks overflow the LDS, several rounds), at both ends of the
    length classes."""
    Wb = 8 if wide else 4
    blk = 128 * Wb
    rng = np.random.default_rng(61 + lead)
    tiny = rng.integers(250, 272, size=300)                    # 16..17 groups of 16 bytes
    med = rng.integers(15 * blk + 1, 16 * blk - Wb, size=200)  # 16 blocks each
    edge = np.array([271, 272, 273, 271, 0, 272] * 20)         # the last one-lane length and the first one past it
    mixed = np.concatenate([tiny[:100], med[:100], edge, tiny[100:], med[100:], rng.integers(0, 16 * blk, size=300)])
    from paper_1609_09840_amd import pmp

    plan = pmp.Plan(0)
    plan.tune(0, 0, 1 << 26, 1)  # few waves: every tile holds 64 such strings
    keys = U.keys_for(wide, 63)
    for name, lengths in (("tiny", tiny), ("medium", med), ("mixed", mixed)):
        rg = W.from_lengths(lengths, 62 + lead, wide, lead=lead)
        say(f"case stage-{name}: wide={wide} count={rg.count} bytes={rg.nbytes}")
        got = U.gpu_hash(rg, keys, 0, plan=plan)
        want = U.oracle_hash(rg, keys, 0)
        assert U.first_mismatch(got, want) is None, (name, U.first_mismatch(got, want))
    assert plan.status() == pmp.PMP_OK
    plan.close()


def test_mad_probe_rate():
    """The multiply-rate probe returns a plausible rate (between 1 T and
    1000 T lane operations per second on one device)."""
    from paper_1609_09840_amd import pmp

    say("case mad probe")
    r = pmp.pmp_probe_mad_rate()
    assert 1e12 < r < 1e15, r


def test_read_probe_rate():
    """The read-bandwidth probe returns a plausible rate for 256 MiB (between
    0.5 and 20 TB/s) and refuses a buffer under 1 MiB."""
    import torch

    from paper_1609_09840_amd import pmp

    say("case read probe")
    b = torch.ones(256 << 20, dtype=torch.uint8, device=U.dev())
    r = pmp.pmp_probe_read_bw(b)
    assert 5e11 < r < 2e13, r
    with pytest.raises(pmp.PmpError):
        pmp.pmp_probe_read_bw(b[: 1 << 19])
