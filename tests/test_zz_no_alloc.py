"""pmp_hash_mixed_noalloc (the static-scratch entry point) through the C ABI:
its outputs equal pmp_hash_mixed's on the same batches, on two calls in a
row (the second with a smaller input, so stale accumulators or status from
the first would show), batches too large for the scratch are refused, and
bad offsets set the caller's status word."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_util as U
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _batches(seed, count, max_len):
    """A PM+32 and a PM+64 batch with long strings (several level-2 nodes,
    so the accumulators are used) and short ones, device-resident."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(seed)
    keep, batches = [], []
    for wide in (False, True):
        lengths = rng.integers(0, max_len, size=count)
        lengths[:3] = [0, 300000 if wide else 200000, 70000]
        rg = W.from_lengths(lengths, seed + wide, wide, lead=int(rng.integers(0, 4)))
        kn = U.keys_for(wide, W.KEY_SEED64 if wide else W.KEY_SEED32)
        buf, off = U.to_dev(rg)
        keys = U.to_dev_keys(kn)
        out = torch.zeros(rg.count, dtype=torch.uint64 if wide else torch.uint32, device=U.dev())
        keep.append((rg, kn, buf, off, keys, out))
        batches.append(pmp.make_batch(wide, buf, off, keys, out))
    return keep, batches


def test_noalloc_equals_mixed_twice():
    import torch

    from paper_1609_09840_amd import pmp

    status = torch.full((1,), -1, dtype=torch.int32, device=U.dev())
    plan = pmp.Plan(0)
    for call, (count, max_len) in enumerate(((3000, 150000), (700, 40000))):  # second call smaller
        keep, batches = _batches(2100 + call, count, max_len)
        say(f"case noalloc call {call}: {sum(k[0].count for k in keep)} strings, {sum(k[0].nbytes for k in keep)} bytes")
        pmp.pmp_hash_mixed_noalloc(batches[0], batches[1], status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        got = [U.as_u64(k[5].cpu().numpy()) for k in keep]
        for k in keep:
            k[5].zero_()
        pmp.pmp_hash_mixed(batches[0], batches[1], plan=plan)
        torch.cuda.synchronize()
        assert plan.status() == pmp.PMP_OK
        for t, k in enumerate(keep):
            want = U.as_u64(k[5].cpu().numpy())
            assert U.first_mismatch(got[t], want) is None, (call, t, U.first_mismatch(got[t], want))
            if call == 1:  # and against the oracle
                assert U.first_mismatch(got[t], U.oracle_hash(k[0], k[1])) is None
    plan.close()


def test_noalloc_refuses_oversized_and_reports_offsets():
    import torch

    from paper_1609_09840_amd import pmp

    status = torch.zeros(1, dtype=torch.int32, device=U.dev())
    keep, batches = _batches(2200, 50, 1000)
    big = pmp.make_batch(False, keep[0][2], keep[0][3], keep[0][4], keep[0][5],
                         buf_bytes=pmp.PMP_NOALLOC_SCRATCH_BYTES * 32)  # claims a huge buffer: refused, nothing runs
    say("case noalloc oversized")
    with pytest.raises(pmp.PmpError) as ei:
        pmp.pmp_hash_mixed_noalloc(big, None, status)
    assert ei.value.code == pmp.PMP_E_NOMEM
    rg = W.from_lengths([10, 20, 30, 40], 2201, False)
    offs = rg.offsets.copy()
    offs[2] = offs[1] - 5  # string 1 runs backwards
    buf = torch.from_numpy(rg.buf).to(U.dev())
    off = torch.from_numpy(offs).to(U.dev())
    out = torch.zeros(4, dtype=torch.uint32, device=U.dev())
    b = pmp.make_batch(False, buf, off, U.to_dev_keys(U.keys_for(False, 1)), out)
    say("case noalloc bad offsets")
    pmp.pmp_hash_mixed_noalloc(b, None, status)
    torch.cuda.synchronize()
    assert int(status.item()) & 1
    # a clean call afterwards: status back to 0 and exact outputs
    pmp.pmp_hash_mixed_noalloc(batches[0], batches[1], status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for k in keep:
        assert U.first_mismatch(U.as_u64(k[5].cpu().numpy()), U.oracle_hash(k[0], k[1])) is None
