"""The configurations at their full sizes, in the launch configuration that
bench.py times (one pmp_hash_mixed launch over every batch of the workload),
checked against the oracle on sampled outputs: every string of 64 KiB or
more (the long-string path and its tree levels), the first and last
strings, and a seeded random sample of the rest. The autotuner's choice of
tiles and launch shape is checked against the default plan's outputs, bit
for bit, over every string."""
from __future__ import annotations

import numpy as np
import pytest

import gpu_util as U
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def sample_idx(rg, n_random, seed, long_bytes=65536):
    rng = np.random.default_rng(seed)
    lens = np.diff(rg.offsets)
    idx = set(rng.choice(rg.count, size=min(n_random, rg.count), replace=False).tolist())
    idx |= set(np.nonzero(lens >= long_bytes)[0].tolist())
    idx |= {0, rg.count - 1}
    return np.array(sorted(idx), dtype=np.int64)


def run_full(wl, seed, n_random=4000):
    import torch

    from paper_1609_09840_amd import pmp

    keep, batches = [], []
    for rg in wl.batches:
        kn = U.keys_for(rg.wide, W.KEY_SEED64 if rg.wide else W.KEY_SEED32)
        buf, off = U.to_dev(rg)
        keys = U.to_dev_keys(kn)
        out = torch.zeros(rg.count, dtype=torch.uint64 if rg.wide else torch.uint32, device=U.dev())
        keep.append((rg, kn, buf, off, keys, out))
        batches.append(pmp.make_batch(rg.wide, buf, off, keys, out))
    pair = (batches + [None])[:2]
    assert len(batches) <= 2
    say(f"case {wl.name} full: {wl.count} strings, {wl.nbytes} bytes, default plan")
    plan = pmp.Plan(0)
    pmp.pmp_hash_mixed(pair[0], pair[1], plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_OK
    first = [U.as_u64(k[5].cpu().numpy()) for k in keep]
    for t, (rg, kn, buf, off, keys, out) in enumerate(keep):
        idx = sample_idx(rg, n_random, seed + t)
        want = U.oracle_hash(U.sample_ragged(rg, idx), kn)
        say(f"  batch {t}: {len(idx)} sampled strings vs the oracle")
        assert U.first_mismatch(first[t][idx], want) is None, (t, U.first_mismatch(first[t][idx], want))
    say(f"case {wl.name} full: autotuned plan")
    tuned = pmp.Plan(0)
    best = pmp.pmp_plan_autotune(tuned, batches)
    say(f"  tuning {best}")
    for k in keep:
        k[5].zero_()
    pmp.pmp_hash_mixed(pair[0], pair[1], plan=tuned)
    torch.cuda.synchronize()
    assert tuned.status() == pmp.PMP_OK
    for t, k in enumerate(keep):
        got = U.as_u64(k[5].cpu().numpy())
        assert U.first_mismatch(got, first[t]) is None, (t, U.first_mismatch(got, first[t]))
    plan.close()
    tuned.close()


def test_c2_full_sampled():
    run_full(W.c2(), 1202)


def test_c3_full_sampled():
    run_full(W.c3(), 1203)


def test_c4_full_sampled():
    run_full(W.c4(), 1204)
