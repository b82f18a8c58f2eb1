#!/usr/bin/env python3
"""Benchmark: GB/s hashed by the batched PM+32/PM+64 path on one MI355X.

A step is one pmp_hash_mixed call (one kernel launch) over a whole batch whose
inputs already sit in HBM. The default workload is the ragged mixed batch:
2^18 strings, lengths round(LogNormal(ln 200, 2.0)) clamped to [1 B, 1 MiB],
each string PM+32 or PM+64 with probability 1/2. Other workloads: --config
c1 | c2 | c3 (see paper_1609_09840_amd/workloads.py).

Prints ONE JSON line. Besides the headline value it carries:
  roofline      algorithmic bytes per launch / mean launch time (HIP events
                on the launch stream) against the 8 TB/s HBM peak, and
                against the read rate a plain streaming kernel reaches on
                the same device (frac_of_achievable); `traffic`
                is the measured HBM bytes per launch from the committed
                rocprofv3 counter summary when it was taken on the current
                kernel source, else null;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload;
  plain_gpu     the one-string-per-launch GPU form on a prefix of the batch;
  incremental   one 1 GiB string hashed through pmp_incr_* in pieces of
                1 MiB, 16 MiB and 256 MiB (both variants), checked equal to
                the batched path's hash of the same string;
  hash_table    pmp_table_build over C2-shaped keys and pmp_table_probe of as
                many queries (half present), with the hashing and table
                kernels timed apart;
  pm128         PM+128 (p = 2^128 + 51) on the C3 shape (64 x 16 MiB) and
                the C2 shape (2^20 strings of 8-256 B).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB/s hashed (PM+32/64, ragged batch) vs roofline & plain GPU; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL = "batch_kernel"
DESCR = {
    "c1": "PM+32, 1024 strings x 64 B",
    "c2": "PM+32, 2^20 strings, lengths uniform in [8, 256] B",
    "c3": "PM+64, 64 strings x 16 MiB",
    "c4": "2^18 strings, lengths round(LogNormal(ln 200, 2.0)) clamped to [1 B, 1 MiB], "
          "half PM+32 / half PM+64, one launch",
}


KERNEL_SOURCES = {
    "pmp_kernels.hip": ("pmp_kernels.hip", "pmp_device.hpp", "pmp_batch.h", "pmp_stage.hpp"),
    "pmp_incr.hip": ("pmp_incr.hip", "pmp_device.hpp", "pmp_batch.h", "pmp_incr.h"),
}


def kernel_source_hash(main: str = "pmp_kernels.hip") -> str:
    """sha256 (first 16 hex digits) of a kernel file and the headers it is
    compiled from, with comments and blank lines removed: edits to comments
    keep it."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[main]:
        with open(os.path.join(ROOT, "paper_1609_09840_amd", "csrc", f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = re.sub(r"//.*$", "", line).rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def read_traffic(config: str, kernel: str = KERNEL, main: str = "pmp_kernels.hip"):
    """HBM bytes per launch from profiles/<kernel>_<config>_counters.json if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash(main):
        return None
    return d.get("hbm_bytes_per_launch")


def algorithmic_bytes(wl) -> int:
    """payload + offsets + outputs + key tables: every byte the path must
    move at least once."""
    tot = 0
    for rg in wl.batches:
        tot += rg.nbytes + 8 * (rg.count + 1) + (8 if rg.wide else 4) * rg.count + 1032 * (8 if rg.wide else 4)
    return tot


def algorithmic_mads(wl) -> int:
    """32x32->64 multiplies of the level-1 sums (Eq. (1), Sec. 6): one per
    PM+32 word, four per PM+64 word, N' = floor(len / W) + 1 words a string.
    The upper levels add under 1 % and are not counted."""
    tot = 0
    for rg in wl.batches:
        W = 8 if rg.wide else 4
        words = int(np.sum(np.diff(rg.offsets) // W + 1))
        tot += words * (4 if rg.wide else 1)
    return tot


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# the paper's own single-core numbers (Haswell i7-4770 at 3.4 GHz, long
# strings), quoted as context only
PAPER_CONTEXT = {"hardware": "Intel Core i7-4770 (Haswell), one core at 3.4 GHz, AVX2",
                 "pm32_bytes_per_cycle": 4.7, "pm64_bytes_per_cycle": 3.3,
                 "pm32_GBps": 16.0, "pm64_GBps": 11.2}


_READ_BW = {}


def achievable_read_gbs(dev) -> float:
    """GB/s a plain streaming read kernel reaches over 1 GiB of device memory
    (pmp_probe_read_bw), measured once per run: the achievable HBM read rate
    the kernels are compared with beside the published 8 TB/s."""
    if "v" not in _READ_BW:
        import torch

        from paper_1609_09840_amd import pmp

        buf = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        _READ_BW["v"] = pmp.pmp_probe_read_bw(buf) / 1e9
        del buf
    return _READ_BW["v"]


def mul_roofline(wl, launch_ms: float) -> dict:
    """The launch's level-1 multiplies per second against the device's own
    v_mad_u64_u32 rate (measured now by the library's probe)."""
    from paper_1609_09840_amd import pmp

    mads = algorithmic_mads(wl)
    peak = pmp.pmp_probe_mad_rate()
    achieved = mads / (launch_ms * 1e-3)
    return {"achieved": round(achieved / 1e12, 3), "peak": round(peak / 1e12, 3), "unit": "T mad32/s",
            "frac": round(achieved / peak, 4), "mads_per_launch": mads}


def launch_spread(step, plan, batches, stream, n: int = 30) -> dict:
    """After the timed region: n launches each between its own HIP events
    (median and p99; the events add a few microseconds to each), and the
    same launch captured once as a hipGraph and replayed n times back to
    back (mean)."""
    import torch

    from paper_1609_09840_amd import pmp

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    g = pmp.Graph(plan, batches)
    try:
        g.launch(stream)  # warm
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        g0.record(stream)
        for _ in range(n):
            g.launch(stream)
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / n
    finally:
        g.close()
    return {"launches": n, "launch_ms_median": round(float(np.median(t)), 5),
            "launch_ms_p99": round(float(np.percentile(t, 99)), 5), "graph_replay_ms": round(graph_ms, 5)}


def setup(wl, dev):
    import torch

    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    keep, batches = [], []
    for rg in wl.batches:
        kn = pmp.pmp_expand_keys64(W.KEY_SEED64) if rg.wide else pmp.pmp_expand_keys32(W.KEY_SEED32)
        buf = torch.from_numpy(rg.buf).to(dev)
        off = torch.from_numpy(rg.offsets).to(dev)
        keys = torch.from_numpy(kn.view(np.int64) if rg.wide else kn.view(np.int32)).to(dev)
        keys = keys.view(torch.uint64 if rg.wide else torch.uint32)
        out = torch.empty(rg.count, dtype=torch.uint64 if rg.wide else torch.uint32, device=dev)
        keep.append((rg, kn, buf, off, keys, out))
        batches.append(pmp.make_batch(rg.wide, buf, off, keys, out))
    while len(batches) < 2:
        batches.append(None)
    return keep, batches


def cpu_baseline(wl, target_cpu_s: float = 12.0):
    """The oracle as it stands, on a prefix of each batch sized for about
    `target_cpu_s` CPU-seconds, all host threads."""
    import oracle
    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    orc = oracle.load()
    threads = min(os.cpu_count() or 1, 64)
    # measure the oracle's per-thread speed on a small prefix first
    probe_bytes, probe_s = 0, 0.0
    for rg in wl.batches:
        kn = pmp.pmp_expand_keys64(W.KEY_SEED64) if rg.wide else pmp.pmp_expand_keys32(W.KEY_SEED32)
        n = int(np.searchsorted(rg.offsets, rg.offsets[0] + (4 << 20)))
        n = max(1, min(n, rg.count))
        t0 = time.perf_counter()
        orc.batch(rg.wide, rg.buf, rg.offsets[: n + 1], kn, oracle.MIXED, nthreads=1)
        probe_s += time.perf_counter() - t0
        probe_bytes += int(rg.offsets[n] - rg.offsets[0])
    per_thread = probe_bytes / max(probe_s, 1e-9)
    budget = per_thread * target_cpu_s  # bytes for ~target_cpu_s CPU-seconds
    share = budget / max(wl.nbytes, 1)
    # a sample smaller than the budget (the whole payload, when it is cheap)
    # is hashed again until about target_cpu_s CPU-seconds have been spent
    tot_bytes, tot_s, nstr, passes = 0, 0.0, 0, 0
    while passes == 0 or tot_s * threads < target_cpu_s:
        for rg in wl.batches:
            kn = pmp.pmp_expand_keys64(W.KEY_SEED64) if rg.wide else pmp.pmp_expand_keys32(W.KEY_SEED32)
            want = rg.offsets[0] + int(share * rg.nbytes)
            n = int(np.searchsorted(rg.offsets, want))
            n = max(1, min(n, rg.count))
            t0 = time.perf_counter()
            orc.batch(rg.wide, rg.buf, rg.offsets[: n + 1], kn, oracle.MIXED, nthreads=threads)
            tot_s += time.perf_counter() - t0
            tot_bytes += int(rg.offsets[n] - rg.offsets[0])
            if passes == 0:
                nstr += n
        passes += 1
    once = tot_bytes // passes
    return {
        "value": round(tot_bytes / tot_s / 1e9, 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "single_thread_GBps": round(per_thread / 1e9, 4),
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "sample": f"first {nstr} strings ({once} bytes, {100.0 * once / wl.nbytes:.1f}% of the payload, "
                  f"both variants in proportion) hashed {passes} time(s), {tot_s:.2f} s wall on {threads} threads",
    }


def other_configs(dev, names=("c1", "c2", "c3"), steps: int = 20) -> dict:
    """The other configurations of the hot path, each in the bench's launch
    form (the library's autotuner on the workload, then one launch per step,
    `steps` back to back between two HIP events on the launch stream):
    C1 in microseconds per batch (median and p99 of launches timed one by
    one, and the mean of back-to-back launches); C2 and C3 in GB/s with the
    roofline fraction of their algorithmic bytes, HBM traffic from their
    committed counters, the plain one-string-per-launch form on a prefix and
    the oracle on a bounded sample."""
    import torch

    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    res = {}
    for name in names:
        wl = W.CONFIGS[name]()
        keep, batches = setup(wl, dev)
        stream = torch.cuda.current_stream()
        plan = pmp.Plan(0)
        plan.reserve(sum(rg.buf.size for rg in wl.batches), wl.count)
        tuning = pmp.pmp_plan_autotune(plan, [b for b in batches if b is not None], stream=stream)

        def step():
            pmp.pmp_hash_mixed(batches[0], batches[1], stream=stream, plan=plan)

        for _ in range(3):
            step()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        if plan.status() != pmp.PMP_OK:
            raise RuntimeError(f"{name}: device status not OK")
        ms = e0.elapsed_time(e1) / steps
        alg = algorithmic_bytes(wl)
        r = {"workload": f"{name}: {DESCR[name]}", "strings": wl.count, "payload_bytes": wl.nbytes,
             "tuning": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in tuning.items()},
             "mean_launch_ms": round(ms, 5)}
        if name == "c1":  # latency-bound: microseconds per batch
            spread = launch_spread(step, plan, [b for b in batches if b is not None], stream)
            r.update({"unit": "us per batch", "value": round(ms * 1e3, 2),
                      "launch_us_median": round(spread["launch_ms_median"] * 1e3, 2),
                      "launch_us_p99": round(spread["launch_ms_p99"] * 1e3, 2),
                      "graph_replay_us": round(spread["graph_replay_ms"] * 1e3, 2),
                      "note": "64 KiB per batch: launch latency, not bandwidth, bounds it"})
        else:
            achieved = alg / (ms * 1e-3) / 1e9
            r.update({"unit": "GB/s", "value": round(wl.nbytes / (ms * 1e-3) / 1e9, 1),
                      "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                                   "traffic": read_traffic(name), "kernel": KERNEL,
                                   "algorithmic_bytes_per_launch": alg,
                                   "frac_of_achievable": round(achieved / achievable_read_gbs(dev), 4)}})
        r["plain_gpu"] = plain_gpu(keep, dev, max_strings=8 if name == "c3" else 4000)
        r["cpu_oracle"] = cpu_baseline(wl, target_cpu_s=3.0)
        res[name] = r
        plan.close()
        del keep, batches
        torch.cuda.empty_cache()
    return res


def plain_gpu(keep, dev, max_strings: int = 4000):
    """The one-string-per-launch GPU form on a prefix of each batch."""
    import torch

    from paper_1609_09840_amd import pmp

    scratch = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
    tot_bytes, tot_s, nstr = 0, 0.0, 0
    share = max_strings / sum(k[0].count for k in keep)
    for rg, kn, buf, off, keys, out in keep:
        n = max(1, min(rg.count, int(rg.count * share)))
        h = rg.offsets[: n + 1]
        o = torch.empty(n, dtype=out.dtype, device=dev)
        pmp.pmp_hash_plain(rg.wide, buf, h, keys, o, 0, scratch)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pmp.pmp_hash_plain(rg.wide, buf, h, keys, o, 0, scratch)
        torch.cuda.synchronize()
        tot_s += time.perf_counter() - t0
        tot_bytes += int(h[-1] - h[0])
        nstr += n
        if not torch.equal(o, out[:n]):
            raise RuntimeError("plain GPU form disagrees with the batched path")
    return {"value": round(tot_bytes / tot_s / 1e9, 4), "unit": "GB/s",
            "sample": f"first {nstr} strings of the batch ({tot_bytes} bytes), same outputs as the batched path"}


def incremental(dev, total: int = 1 << 30, pieces=(1 << 20, 16 << 20, 256 << 20), reps: int = 3) -> dict:
    """One string of `total` bytes appended in equal pieces, then a digest.
    HIP events on the object's stream: one pair around the appends of a pass
    (per-append time = its share; an append is one launch), one more after
    the digest; `reps` passes after a warm one, each after a reset. The digest
    must equal pmp_hash32/64 of the string. `roofline`: the largest pieces'
    append rate against the HBM peak (algorithmic bytes = the piece)."""
    import torch

    from paper_1609_09840_amd import pmp

    g = torch.Generator(device=dev)
    g.manual_seed(909)
    data = torch.randint(0, 256, (total,), dtype=torch.uint8, device=dev, generator=g)
    off = torch.tensor([0, total], dtype=torch.int64, device=dev)
    res = {"string_bytes": total, "unit": "GB/s", "runs": []}
    for wide in (False, True):
        kn = pmp.pmp_expand_keys64(2) if wide else pmp.pmp_expand_keys32(1)
        keys = torch.from_numpy(kn.view(np.int64) if wide else kn.view(np.int32)).to(dev)
        keys = keys.view(torch.uint64 if wide else torch.uint32)
        ref = (pmp.pmp_hash64 if wide else pmp.pmp_hash32)(data, off, keys)
        h = pmp.Incr(wide, keys)
        h.reserve(max(pieces))
        for piece in pieces:
            n_app = -(-total // piece)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            t_app = t_all = 0.0
            for r in range(reps + 1):
                h.reset()
                ev[0].record()
                for o in range(0, total, piece):
                    h.append(data[o:o + piece])
                ev[1].record()
                d = h.digest()
                ev[2].record()
                ev[2].synchronize()
                if r:  # the first pass warms up
                    t_app += ev[0].elapsed_time(ev[1]) / reps
                    t_all += ev[0].elapsed_time(ev[2]) / reps
                if not torch.equal(d, ref):
                    raise RuntimeError("incremental digest disagrees with the batched path")
            res["runs"].append({"variant": "PM+64" if wide else "PM+32", "piece_bytes": piece, "appends": n_app,
                                "append_us": round(t_app * 1e3 / n_app, 2),
                                "append_GBps": round(total / (t_app * 1e-3) / 1e9, 1),
                                "digest_us": round((t_all - t_app) * 1e3, 2),
                                "value": round(total / (t_all * 1e-3) / 1e9, 1)})
        h.close()
    big = [r for r in res["runs"] if r["piece_bytes"] == max(pieces)]
    best = max(big, key=lambda r: r["append_GBps"])
    res["roofline"] = {"bound": "hbm", "kernel": "incr_blocks (one append)",
                       "variant": best["variant"], "piece_bytes": best["piece_bytes"],
                       "achieved": best["append_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(best["append_GBps"] / HBM_PEAK_GBS, 4),
                       "traffic": read_traffic("256mib_" + ("pm64" if best["variant"] == "PM+64" else "pm32"),
                                               "incr_blocks", "pmp_incr.hip"),
                       "achievable_read_GBps": round(achievable_read_gbs(dev), 1),
                       "frac_of_achievable": round(best["append_GBps"] / achievable_read_gbs(dev), 4)}
    return res


def gather_strings(buf: np.ndarray, offsets: np.ndarray, idx: np.ndarray):
    """The strings idx of a ragged set, back to back (vectorized)."""
    lens = offsets[idx + 1] - offsets[idx]
    off = np.zeros(len(idx) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    pos = np.repeat(offsets[idx] - off[:-1], lens) + np.arange(off[-1], dtype=np.int64)
    return buf[pos], off


def hash_table(dev, nkeys: int = 1 << 20, nbuckets: int = 1 << 20, reps: int = 5) -> dict:
    """Build a table over C2-shaped keys (PM+32, lengths uniform in [8, 256])
    and probe as many queries: even-numbered ones copy a random key, odd ones
    are fresh strings. HIP events: whole build and probe calls, and the
    hashing launches alone (pmp_hash32 on the same batches), over `reps`
    calls after a warm one. Every hit is checked to carry the query's hash
    and length, and the hit count to be the number of copied queries."""
    import torch

    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    rng = np.random.default_rng(606)
    keys_rg = W.from_lengths(rng.integers(8, 257, nkeys), 607, False)
    fresh = W.from_lengths(rng.integers(8, 257, nkeys), 608, False)
    # query q copies a random key when q is even, else it is fresh string q: one
    # gather from the keys and fresh strings laid end to end
    pool = np.concatenate([keys_rg.buf, fresh.buf])
    pool_off = np.concatenate([keys_rg.offsets[:-1], fresh.offsets + keys_rg.offsets[-1]])
    take_copy = np.arange(nkeys) % 2 == 0
    idx = np.where(take_copy, rng.integers(0, nkeys, nkeys), nkeys + np.arange(nkeys))
    qbuf, qoff = gather_strings(pool, pool_off, idx)
    lens = np.diff(qoff)
    kn = pmp.pmp_expand_keys32(1)
    keys = torch.from_numpy(kn.view(np.int32)).to(dev).view(torch.uint32)
    dk = torch.from_numpy(keys_rg.buf).to(dev)
    dko = torch.from_numpy(keys_rg.offsets).to(dev)
    dq = torch.from_numpy(qbuf).to(dev)
    dqo = torch.from_numpy(qoff).to(dev)
    plan = pmp.Plan(0)
    plan.reserve(max(dk.numel(), dq.numel()), nkeys)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        ev[0].record()
        for _ in range(reps):
            r = fn()
        ev[1].record()
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / reps, r

    t = pmp.Table(False, dk, dko, keys, nbuckets, plan=plan)
    qh = torch.empty(nkeys, dtype=torch.uint32, device=dev)
    res = torch.empty(nkeys, dtype=torch.int64, device=dev)
    build_ms, _ = timed(lambda: pmp.Table(False, dk, dko, keys, nbuckets, plan=plan))
    probe_ms, _ = timed(lambda: t.probe(dq, dqo, out=res, qhashes=qh))
    hk_ms, _ = timed(lambda: pmp.pmp_hash32(dk, dko, keys, out=t.hashes, plan=plan))
    hq_ms, _ = timed(lambda: pmp.pmp_hash32(dq, dqo, keys, out=qh, plan=plan))
    torch.cuda.synchronize()
    got = res.cpu().numpy()
    kh = t.hashes.cpu().numpy()
    qhn = qh.cpu().numpy()
    hit = got >= 0
    if hit.sum() != take_copy.sum() or not np.array_equal(kh[got[hit]], qhn[hit]) or \
            not np.array_equal(np.diff(keys_rg.offsets)[got[hit]], lens[hit]):
        raise RuntimeError("hash-table probe results fail their checks")
    kb, qb = int(keys_rg.offsets[-1]), int(qoff[-1])
    return {"keys": nkeys, "buckets": nbuckets, "key_bytes": kb, "queries": nkeys, "query_bytes": qb,
            "hits": int(hit.sum()),
            "build_ms": round(build_ms, 4), "build_Mkeys_per_s": round(nkeys / build_ms / 1e3, 1),
            "build_GBps": round(kb / (build_ms * 1e-3) / 1e9, 1), "build_hash_ms": round(hk_ms, 4),
            "probe_ms": round(probe_ms, 4), "probe_Mqueries_per_s": round(nkeys / probe_ms / 1e3, 1),
            "probe_GBps": round(qb / (probe_ms * 1e-3) / 1e9, 1), "probe_hash_ms": round(hq_ms, 4),
            "note": "GB/s = key or query payload bytes per second of the whole call (hashing + table kernels)"}


def pm128(dev, reps: int = 5) -> dict:
    """pmp_hash128 on two shapes with device-resident seeded bytes; HIP events
    around `reps` back-to-back calls after a warm one (a call is seven
    launches: counts, a three-launch scan, short strings, nodes, upper
    levels)."""
    import torch

    from paper_1609_09840_amd import pmp

    kt = torch.from_numpy(pmp.pmp_expand_keys128(1).view(np.int64)).to(dev).view(torch.uint64)
    g = torch.Generator(device=dev)
    g.manual_seed(1280)
    rng = np.random.default_rng(1281)
    shapes = {"c3-shaped: 64 x 16 MiB": np.full(64, 16 << 20, np.int64),
              "c2-shaped: 2^20 strings, lengths uniform in [8, 256] B": rng.integers(8, 257, 1 << 20)}
    runs = []
    for name, lens in shapes.items():
        off = np.zeros(len(lens) + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        buf = torch.randint(0, 256, (int(off[-1]),), dtype=torch.uint8, device=dev, generator=g)
        doff = torch.from_numpy(off).to(dev)
        out = torch.empty(2 * len(lens), dtype=torch.uint64, device=dev)
        scratch = torch.empty(int(pmp._lib.pmp_hash128_scratch_bytes(len(lens), buf.numel())), dtype=torch.uint8,
                              device=dev)
        pmp.pmp_hash128(buf, doff, kt, out=out, scratch=scratch)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pmp.pmp_hash128(buf, doff, kt, out=out, scratch=scratch)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = int(off[-1]) / (ms * 1e-3) / 1e9
        runs.append({"workload": name, "payload_bytes": int(off[-1]), "ms": round(ms, 4), "value": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
        del buf, scratch
    return {"unit": "GB/s", "runs": runs}


def serving_sweep(dev, pool_size: int = 48, points: int = 8, seed: int = 505, per_launch: int = 16,
                  sat_passes: int = 8):
    """Serving workload: Poisson arrivals of requests of 1..4096 strings with
    lengths log-uniform in [16 B, 64 KiB], variant per request, payloads
    pre-staged in a device-resident pool (the device batching is measured, not
    PCIe). The saturation rate is measured first (the pool submitted
    `sat_passes` times over, all at once, at most `per_launch` requests per
    launch so that the lanes overlap); then `points` rates from 0.1x to 1.2x
    of it, geometric."""
    import torch

    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    rng = np.random.default_rng(seed)
    pool, reqs = [], []
    for k in range(pool_size):
        rg = W.c5_request(rng, 5000 + k)
        buf = torch.from_numpy(rg.buf).to(dev)
        off = torch.from_numpy(rg.offsets).to(dev)
        out = torch.empty(rg.count, dtype=torch.uint64 if rg.wide else torch.uint32, device=dev)
        pool.append((rg, buf, off, out))
        reqs.append(pmp.Server.request(rg.wide, buf, off, out))
    mean_bytes = float(np.mean([p[0].nbytes for p in pool]))
    k32 = torch.from_numpy(pmp.pmp_expand_keys32(W.KEY_SEED32).view(np.int32)).to(dev).view(torch.uint32)
    k64 = torch.from_numpy(pmp.pmp_expand_keys64(W.KEY_SEED64).view(np.int64)).to(dev).view(torch.uint64)
    # one request alone: host wall time of one launch and its completion (the floor of a request's latency)
    plan = pmp.Plan(0)
    stream = torch.cuda.current_stream()
    alone = []
    for rep in range(3):
        for rg, buf, off, out in pool:
            b = pmp.make_batch(rg.wide, buf, off, k64 if rg.wide else k32, out)
            t0 = time.perf_counter()
            pmp.pmp_hash_many([b], plan=plan, stream=stream)
            stream.synchronize()
            if rep:
                alone.append((time.perf_counter() - t0) * 1e3)
    plan.close()
    budget = 1 << 30
    srv = pmp.Server(k32, k64, device=0, lanes=4, lane_bytes=0, max_requests_per_batch=per_launch,
                     max_inflight_bytes=budget, idle_spin_us=200)
    try:
        srv.replay(reqs, np.zeros(len(reqs)))  # warm-up
        srv.reset_stats()
        srv.replay(reqs * sat_passes, np.zeros(sat_passes * len(reqs)))
        st = srv.stats()
        sat_rps = st["completed"] / (st["span_us"] * 1e-6)
        rows = []
        for rate in sat_rps * np.geomspace(0.1, 1.2, points):
            n = int(min(max(40, rate * 1.0), 400))
            gaps = rng.exponential(1e6 / rate, size=n)
            arrivals = np.cumsum(gaps) - gaps[0]
            srv.reset_stats()
            lat = srv.replay([reqs[i % len(reqs)] for i in range(n)], arrivals)
            st = srv.stats()
            rows.append({"offered_rps": round(float(rate), 2), "requests": n,
                         "achieved_GBps": round(st["bytes"] / (st["span_us"] * 1e-6) / 1e9, 2),
                         "p50_ms": round(float(np.percentile(lat, 50)) / 1e3, 4),
                         "p99_ms": round(float(np.percentile(lat, 99)) / 1e3, 4),
                         "requests_per_launch": round(n / max(1, st["batches"]), 2)})
        if srv.status() != pmp.PMP_OK:
            raise RuntimeError("serving: device status not OK")
    finally:
        srv.close()
    host = serving_host(pool, k32, k64, per_launch)
    return {"mean_request_bytes": round(mean_bytes), "saturation_rps": round(float(sat_rps), 2),
            "saturation_GBps": round(sat_rps * mean_bytes / 1e9, 2), "lanes": 4,
            "max_requests_per_launch": per_launch, "max_inflight_bytes": budget, "idle_spin_us": 200,
            "alone_ms_p50": round(float(np.percentile(alone, 50)), 4),
            "alone_ms_p99": round(float(np.percentile(alone, 99)), 4),
            "alone_note": "one request of the pool hashed by itself: host wall time of its launch and completion",
            "payload": "device-resident pool of %d requests" % pool_size, "sweep": rows,
            "host_staged": host}


def serving_host(pool, k32, k64, per_launch: int, passes: int = 2) -> dict:
    """The same requests given as host arrays: the server copies each into a
    lane's pinned arena and over PCIe, hashes it, and copies the outputs
    back. All submitted at once, `passes` times over; outputs checked equal
    to the device-resident results. PCIe-bound: reported apart, never as the
    headline value."""
    import torch

    from paper_1609_09840_amd import pmp

    reqs, outs, want = [], [], []
    for rg, buf, off, out in pool:
        o = np.zeros(rg.count, dtype=np.uint64 if rg.wide else np.uint32)
        outs.append(o)
        want.append(out.cpu().numpy())
        reqs.append(pmp.Server.request(rg.wide, rg.buf, rg.offsets, o))
    need = max(rg.nbytes + 16 * (rg.count + 1) for rg, _, _, _ in pool)
    lane_bytes = int(need * 1.25) + (1 << 20)
    srv = pmp.Server(k32, k64, device=0, lanes=2, lane_bytes=lane_bytes, max_requests_per_batch=per_launch,
                     reserve_bytes=64 << 20)
    try:
        srv.replay(reqs, np.zeros(len(reqs)))  # warm-up
        for o, w in zip(outs, want):
            if not np.array_equal(o, w):
                raise RuntimeError("host-staged serving disagrees with the device-resident results")
        srv.reset_stats()
        lat = srv.replay(reqs * passes, np.zeros(passes * len(reqs)))
        st = srv.stats()
        if srv.status() != pmp.PMP_OK:
            raise RuntimeError("host-staged serving: device status not OK")
    finally:
        srv.close()
    span = st["span_us"] * 1e-6
    return {"requests": int(st["completed"]), "lanes": 2, "lane_bytes": lane_bytes,
            "rps": round(st["completed"] / span, 2), "GBps_incl_pcie": round(st["bytes"] / span / 1e9, 2),
            "p50_ms": round(float(np.percentile(lat, 50)) / 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) / 1e3, 3),
            "note": "payload and outputs cross PCIe (host arrays staged through pinned arenas)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c4", choices=sorted(DESCR))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain GPU form")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1, C2 and C3 passes")
    ap.add_argument("--configs-only", action="store_true", help="only run the C1, C2 and C3 passes")
    ap.add_argument("--g32", type=int, default=0, help="lanes per block, PM+32 (0: default)")
    ap.add_argument("--g64", type=int, default=0, help="lanes per block, PM+64 (0: default)")
    ap.add_argument("--waves-per-cu", type=int, default=0, help="waves per CU (0: as many as stay resident)")
    ap.add_argument("--alpha", type=int, default=0, help="per-string work weight in bytes (0: default)")
    ap.add_argument("--shares", type=int, default=0, help="shares of the work per wave (0: default)")
    ap.add_argument("--no-incr", action="store_true", help="skip the incremental (one string in pieces) pass")
    ap.add_argument("--incr-only", action="store_true",
                    help="only run the incremental pass and print its JSON (for profiling its kernels)")
    ap.add_argument("--no-table", action="store_true", help="skip the hash-table pass")
    ap.add_argument("--no-pm128", action="store_true", help="skip the PM+128 pass")
    ap.add_argument("--pm128-only", action="store_true", help="only run the PM+128 pass and print its JSON")
    ap.add_argument("--table-only", action="store_true", help="only run the hash-table pass and print its JSON")
    ap.add_argument("--serve-only", action="store_true", help="only run the serving sweep and print its JSON")
    ap.add_argument("--incr-pieces", default="1048576,16777216,268435456",
                    help="piece sizes of the incremental pass, in bytes, comma-separated")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1609_09840_amd import pmp
    from paper_1609_09840_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.randint(0, 255, (args.calibrate_copy,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "launches": 5}), flush=True)
        return
    incr_pieces = tuple(int(x) for x in args.incr_pieces.split(",") if x)
    if args.pm128_only:
        print(json.dumps({"pm128": pm128(dev)}), flush=True)
        return
    if args.table_only:
        print(json.dumps({"hash_table": hash_table(dev)}), flush=True)
        return
    if args.configs_only:
        print(json.dumps({"configs": other_configs(dev)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_sweep(dev)}), flush=True)
        return
    if args.incr_only:
        print(json.dumps({"incremental": incremental(dev, pieces=incr_pieces)}), flush=True)
        return
    wl = W.CONFIGS[args.config]()
    keep, batches = setup(wl, dev)
    plan = pmp.Plan(0)
    plan.reserve(sum(rg.buf.size for rg in wl.batches), wl.count)
    stream = torch.cuda.current_stream()
    manual = bool(args.g32 or args.g64 or args.waves_per_cu or args.alpha or args.shares)
    if manual:
        if args.g32:
            plan.set_tile(False, args.g32)
        if args.g64:
            plan.set_tile(True, args.g64)
        plan.tune(args.waves_per_cu, args.alpha, 0, args.shares)
        tuning = {"source": "command line", "g32": plan_g(args.g32), "g64": plan_g(args.g64, True),
                  "alpha": args.alpha or 768, "waves_per_cu": args.waves_per_cu, "shares_per_wave": args.shares or 1}
    else:  # the library's autotuner, on this workload, before the warm-up
        tuning = pmp.pmp_plan_autotune(plan, [b for b in batches if b is not None], stream=stream)
        tuning = {"source": "pmp_plan_autotune", **{k: (round(v, 4) if isinstance(v, float) else v)
                                                    for k, v in tuning.items()}}

    def step():
        pmp.pmp_hash_mixed(batches[0], batches[1], stream=stream, plan=plan)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if plan.status() != pmp.PMP_OK:
        raise RuntimeError("device status not OK after warmup")

    # one event pair on the launch stream around the whole timed region (an
    # event between launches would itself add a few microseconds per step)
    e_start = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record(stream)
    for _ in range(args.steps):
        step()
    e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = e_start.elapsed_time(e_end) / args.steps  # mean launch, back to back
    if plan.status() != pmp.PMP_OK:
        raise RuntimeError("device status not OK after the timed steps")

    payload = wl.nbytes
    value = payload * args.steps / wall / 1e9
    alg = algorithmic_bytes(wl)
    achieved = alg / (launch_ms * 1e-3) / 1e9
    traffic = read_traffic(args.config)
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded PCG64 bytes and lengths)",
        "config": {
            "workload": f"{args.config}: {DESCR[args.config]}",
            "strings": wl.count,
            "payload_bytes": payload,
            "tuning": tuning,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": KERNEL,
            "algorithmic_bytes_per_launch": alg,
            "mean_launch_ms": round(launch_ms, 5),
            "achievable_read_GBps": round(achievable_read_gbs(dev), 1),
            "frac_of_achievable": round(achieved / achievable_read_gbs(dev), 4),
        },
        "mul_roofline": mul_roofline(wl, launch_ms),
        "paper_context": PAPER_CONTEXT,
    }
    rec["launch_spread"] = launch_spread(step, plan, [b for b in batches if b is not None], stream)
    if plan.status() != pmp.PMP_OK:
        raise RuntimeError("device status not OK after the spread pass")
    if not args.no_plain:
        rec["plain_gpu"] = plain_gpu(keep, dev)
    if not args.no_configs:
        rec["configs"] = other_configs(dev)
    if not args.no_serve:
        rec["serving"] = serving_sweep(dev)
    if not args.no_incr:
        rec["incremental"] = incremental(dev, pieces=incr_pieces)
    if not args.no_table:
        rec["hash_table"] = hash_table(dev)
    if not args.no_pm128:
        rec["pm128"] = pm128(dev)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(rec), flush=True)


def plan_g(g: int, wide: bool = False) -> int:
    return g if g else 8  # the plan default: 8 lanes per block for both variants


if __name__ == "__main__":
    main()
