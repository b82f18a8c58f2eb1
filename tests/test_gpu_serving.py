"""Many batches in one launch, and the serving loop: every output equals the
oracle's and the output of the same request hashed alone, bit for bit.

Requests follow the serving workload: 1..4096 strings per request, lengths
log-uniform in [16 B, 64 KiB], variant drawn per request (scaled down in
count where a test only needs a mix)."""
from __future__ import annotations

import threading

import numpy as np
import pytest

import gpu_util as U
from paper_1609_09840_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_of(rg, flags=0):
    return U.oracle_hash(rg, U.keys_for(rg.wide, W.KEY_SEED64 if rg.wide else W.KEY_SEED32), flags)


def out_dtype(wide, flags):
    import torch

    if flags & 2:
        return torch.uint64
    return torch.uint64 if wide else torch.uint32


def out_len(rg, flags):
    return rg.count * (2 if (rg.wide and flags & 2) else 1)


def small_request(rng, data_seed, max_count=256):
    count = int(rng.integers(1, max_count + 1))
    lengths = np.rint(np.exp(rng.uniform(np.log(16.0), np.log(65536.0), size=count))).astype(np.int64)
    return W.from_lengths(lengths, data_seed, bool(rng.random() < 0.5))


def test_hash_many_vs_oracle():
    """Seven batches (both variants, all output modes, an empty one, offsets
    that do not start at 0) in one launch, then three in a second launch on
    the same plan."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(501)
    specs = []
    for k in range(7):
        wide = bool(k % 2)
        flags = k % 3
        lengths = rng.integers(0, 40000, size=int(rng.integers(1, 300)))
        if k == 4:
            lengths = np.zeros(0, np.int64)
        specs.append((W.from_lengths(lengths, 510 + k, wide, lead=k), flags))
    plan = pmp.Plan(0)
    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    for rounds in ([0, 1, 2, 3, 4, 5, 6], [6, 3, 0]):
        say(f"case hash_many batches={rounds}")
        keep, batches = [], []
        for k in rounds:
            rg, flags = specs[k]
            buf, off = U.to_dev(rg)
            out = torch.zeros(out_len(rg, flags), dtype=out_dtype(rg.wide, flags), device=U.dev())
            keep.append((rg, flags, buf, off, out))
            batches.append(pmp.make_batch(rg.wide, buf, off, k64 if rg.wide else k32, out, flags))
        pmp.pmp_hash_many(batches, plan=plan)
        torch.cuda.synchronize()
        assert plan.status() == pmp.PMP_OK
        for rg, flags, buf, off, out in keep:
            got = U.as_u64(out.cpu().numpy())
            want = oracle_of(rg, flags)
            assert U.first_mismatch(got, want) is None, U.first_mismatch(got, want)
    plan.close()


def _server(lanes=2, lane_bytes=64 << 20, **kw):
    from paper_1609_09840_amd import pmp

    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    return pmp.Server(k32, k64, device=0, lanes=lanes, lane_bytes=lane_bytes, **kw)


def test_server_device_requests_alone_equals_mix():
    """Poisson arrivals fast enough to overlap; each request's output is the
    oracle's and the same as that request hashed alone with pmp_hash32/64."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(601)
    reqs, keep = [], []
    for k in range(24):
        rg = W.c5_request(rng, 610 + k) if k % 3 == 0 else small_request(rng, 610 + k)
        buf, off = U.to_dev(rg)
        out = torch.zeros(rg.count, dtype=out_dtype(rg.wide, 0), device=U.dev())
        keep.append((rg, buf, off, out))
        reqs.append(pmp.Server.request(rg.wide, buf, off, out))
    arrivals = np.cumsum(rng.exponential(300.0, size=len(reqs)))  # mean gap 300 us
    say(f"case server device-resident: {len(reqs)} requests, {sum(k[0].nbytes for k in keep)} bytes")
    srv = _server(lanes=3)
    lat = srv.replay(reqs, arrivals)
    assert srv.status() == pmp.PMP_OK
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs) and np.all(lat > 0)
    srv.close()
    for rg, buf, off, out in keep:
        got = U.as_u64(out.cpu().numpy())
        alone = U.gpu_hash(rg, U.keys_for(rg.wide, W.KEY_SEED64 if rg.wide else W.KEY_SEED32), 0, buf=buf, off=off)
        want = oracle_of(rg)
        assert U.first_mismatch(got, alone) is None, ("mix vs alone", U.first_mismatch(got, alone))
        assert U.first_mismatch(got, want) is None, ("mix vs oracle", U.first_mismatch(got, want))


def test_server_48_full_c5_requests_alone_equals_mix():
    """48 requests drawn exactly as the serving workload draws them (1..4096
    strings, 16 B..64 KiB), device-resident, arriving as a Poisson stream
    fast enough that launches overlap on four lanes: each output equals the
    same request hashed alone and the oracle, bit for bit."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(1601)
    reqs, keep = [], []
    for k in range(48):
        rg = W.c5_request(rng, 1610 + k)
        buf, off = U.to_dev(rg)
        out = torch.zeros(rg.count, dtype=out_dtype(rg.wide, 0), device=U.dev())
        keep.append((rg, buf, off, out))
        reqs.append(pmp.Server.request(rg.wide, buf, off, out))
    arrivals = np.cumsum(rng.exponential(20.0, size=len(reqs)))  # mean gap 20 us: many in flight
    say(f"case server 48 full C5 requests: {sum(k[0].nbytes for k in keep)} bytes")
    srv = _server(lanes=4, lane_bytes=0, max_requests_per_batch=16)
    lat = srv.replay(reqs, arrivals)
    assert srv.status() == pmp.PMP_OK
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs) and np.all(lat > 0)
    srv.close()
    for i, (rg, buf, off, out) in enumerate(keep):
        got = U.as_u64(out.cpu().numpy())
        alone = U.gpu_hash(rg, U.keys_for(rg.wide, W.KEY_SEED64 if rg.wide else W.KEY_SEED32), 0, buf=buf, off=off)
        want = oracle_of(rg)
        assert U.first_mismatch(got, alone) is None, (i, "mix vs alone", U.first_mismatch(got, alone))
        assert U.first_mismatch(got, want) is None, (i, "mix vs oracle", U.first_mismatch(got, want))


def test_server_bad_offsets_fail_only_their_request():
    """A device-resident request with decreasing offsets, submitted with good
    ones so that they share a launch: only it fails (PMP_E_OFFSETS), the
    others, and the requests after it on the same lane, match the oracle.
    A host request with bad offsets is refused at submit."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(1701)
    srv = _server(lanes=1, lane_bytes=8 << 20, max_requests_per_batch=8)
    keep, tickets = [], []
    bad = W.from_lengths([10, 20, 30, 40], 1702, False)
    offs = bad.offsets.copy()
    offs[2] = offs[1] - 5  # string 1 runs backwards
    bad_buf = torch.from_numpy(bad.buf).to(U.dev())
    bad_off = torch.from_numpy(offs).to(U.dev())
    bad_out = torch.zeros(4, dtype=torch.uint32, device=U.dev())
    say("case server bad offsets: 1 bad request among 11")
    for k in range(11):
        if k == 3:
            tickets.append(srv.submit(pmp.Server.request(False, bad_buf, bad_off, bad_out)))
            keep.append(None)
            continue
        rg = small_request(rng, 1710 + k, max_count=128)
        buf, off = U.to_dev(rg)
        out = torch.zeros(rg.count, dtype=out_dtype(rg.wide, 0), device=U.dev())
        keep.append((rg, buf, off, out))
        tickets.append(srv.submit(pmp.Server.request(rg.wide, buf, off, out)))
    for k, t in enumerate(tickets):
        if k == 3:
            with pytest.raises(pmp.PmpError) as ei:
                srv.wait(t)
            assert ei.value.code == pmp.PMP_E_OFFSETS
        else:
            assert srv.wait(t) == pmp.PMP_OK
    hbad = W.from_lengths([10, 20], 1703, False)
    hoffs = hbad.offsets.copy()
    hoffs[-1] = hbad.buf.size + 1  # past the payload
    with pytest.raises(pmp.PmpError) as ei:
        srv.submit(pmp.Server.request(False, hbad.buf, hoffs, np.zeros(2, np.uint32)))
    assert ei.value.code == pmp.PMP_E_OFFSETS
    st = srv.stats()
    say(f"stats {st}")
    assert st["failed"] == 1 and st["completed"] == 10
    assert srv.status() == pmp.PMP_OK
    srv.close()
    for item in keep:
        if item is None:
            continue
        rg, buf, off, out = item
        want = oracle_of(rg)
        assert U.first_mismatch(U.as_u64(out.cpu().numpy()), want) is None


def test_server_inflight_budget():
    """Device-resident requests admitted against an in-flight byte budget:
    one larger than the budget is refused at submit; the rest complete
    exactly while never more than the budget is on the device at once."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(1801)
    budget = 2 << 20
    srv = _server(lanes=4, lane_bytes=0, max_requests_per_batch=16, max_inflight_bytes=budget)
    big = W.from_lengths([budget + 1], 1802, False)
    bbuf, boff = U.to_dev(big)
    bout = torch.zeros(1, dtype=torch.uint32, device=U.dev())
    with pytest.raises(pmp.PmpError) as ei:
        srv.submit(pmp.Server.request(False, bbuf, boff, bout))
    assert ei.value.code == pmp.PMP_E_NOMEM
    reqs, keep = [], []
    for k in range(30):
        rg = small_request(rng, 1810 + k, max_count=64)
        buf, off = U.to_dev(rg)
        out = torch.zeros(rg.count, dtype=out_dtype(rg.wide, 0), device=U.dev())
        keep.append((rg, buf, off, out))
        reqs.append(pmp.Server.request(rg.wide, buf, off, out))
    say(f"case server budget: {len(reqs)} requests, {sum(k[0].nbytes for k in keep)} bytes, budget {budget}")
    srv.replay(reqs, np.zeros(len(reqs)))
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs) and st["rejected"] == 1
    assert srv.status() == pmp.PMP_OK
    srv.close()
    for rg, buf, off, out in keep:
        assert U.first_mismatch(U.as_u64(out.cpu().numpy()), oracle_of(rg)) is None


def test_server_host_requests_and_admission():
    """Host requests are staged through the lane arenas; one larger than an
    arena is refused at submit; the rest complete with the oracle's values."""
    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(701)
    lane_bytes = 4 << 20
    srv = _server(lanes=2, lane_bytes=lane_bytes, max_requests_per_batch=8)
    big = W.from_lengths([lane_bytes], 702, False)
    big_out = np.zeros(1, np.uint32)
    say("case server admission: request larger than the arena")
    with pytest.raises(pmp.PmpError) as ei:
        srv.submit(pmp.Server.request(False, big.buf, big.offsets, big_out))
    assert ei.value.code == pmp.PMP_E_NOMEM
    reqs, keep = [], []
    for k in range(40):
        rg = small_request(rng, 710 + k, max_count=64)
        flags = int(rng.integers(0, 3))
        n = out_len(rg, flags)
        out = np.zeros(n, np.uint64 if (rg.wide or flags & 2) else np.uint32)
        keep.append((rg, flags, out))
        reqs.append(pmp.Server.request(rg.wide, rg.buf, rg.offsets, out, flags))
    say(f"case server host requests: {len(reqs)} requests")
    lat = srv.replay(reqs, np.cumsum(rng.exponential(100.0, size=len(reqs))))
    assert srv.status() == pmp.PMP_OK
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(reqs) and st["rejected"] == 1 and np.all(lat > 0)
    srv.close()
    for rg, flags, out in keep:
        want = oracle_of(rg, flags)
        assert U.first_mismatch(U.as_u64(out), want) is None, U.first_mismatch(U.as_u64(out), want)


def test_server_submit_from_threads():
    """Four host threads submit and wait concurrently on one server."""
    from paper_1609_09840_amd import pmp

    srv = _server(lanes=2, lane_bytes=16 << 20)
    results, errors = {}, []

    def worker(t):
        try:
            rng = np.random.default_rng(800 + t)
            for k in range(10):
                rg = small_request(rng, 8000 + 100 * t + k, max_count=32)
                out = np.zeros(rg.count, np.uint64 if rg.wide else np.uint32)
                tk = srv.submit(pmp.Server.request(rg.wide, rg.buf, rg.offsets, out), keep=(rg, out))
                assert srv.wait(tk) == pmp.PMP_OK
                results[(t, k)] = (rg, out)
        except Exception as e:  # reported below
            errors.append(repr(e))

    say("case server threads: 4 x 10 requests")
    th = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not errors, errors
    assert srv.status() == pmp.PMP_OK
    srv.close()
    assert len(results) == 40
    for rg, out in results.values():
        want = oracle_of(rg)
        assert U.first_mismatch(U.as_u64(out), want) is None


def _batches_for(specs, k32, k64):
    import torch

    from paper_1609_09840_amd import pmp

    keep, batches = [], []
    for rg, flags in specs:
        buf, off = U.to_dev(rg)
        out = torch.zeros(out_len(rg, flags), dtype=out_dtype(rg.wide, flags), device=U.dev())
        keep.append((rg, flags, buf, off, out))
        batches.append(pmp.make_batch(rg.wide, buf, off, k64 if rg.wide else k32, out, flags))
    return keep, batches


@pytest.mark.parametrize("nb", [2, 5])
def test_graph_replays(nb):
    """A captured launch replayed several times, with eager work and new data
    in the same buffers between replays; every replay matches the oracle."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(900 + nb)
    specs = []
    for k in range(nb):
        lengths = rng.integers(0, 70000, size=int(rng.integers(1, 200)))
        specs.append((W.from_lengths(lengths, 910 + k, bool(k % 2)), k % 3))
    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    keep, batches = _batches_for(specs, k32, k64)
    plan = pmp.Plan(0)
    say(f"case graph nb={nb}")
    g = pmp.Graph(plan, batches)
    stream = torch.cuda.current_stream()
    for rep in range(3):
        if rep:  # new bytes in the same buffers, and some eager work between replays
            for rg, flags, buf, off, out in keep:
                rg.buf[:] = np.frombuffer(np.random.default_rng(rep * 100 + rg.count).bytes(rg.buf.size), np.uint8)
                buf.copy_(torch.from_numpy(rg.buf))
                out.zero_()
            _ = torch.arange(1000, device=U.dev()).sum().item()
        g.launch(stream)
        torch.cuda.synchronize()
        assert plan.status() == pmp.PMP_OK
        for rg, flags, buf, off, out in keep:
            got = U.as_u64(out.cpu().numpy())
            want = oracle_of(rg, flags)
            assert U.first_mismatch(got, want) is None, (rep, U.first_mismatch(got, want))
    g.close()
    plan.close()


def test_autotune_keeps_results():
    """The autotuner picks a compiled setting and the outputs stay exact."""
    import torch

    from paper_1609_09840_amd import pmp

    lengths = W.c4_lengths(4096, seed=931)
    lens, wide = lengths
    specs = [(W.from_lengths(lens[~wide], 932, False), 0), (W.from_lengths(lens[wide], 933, True), 0)]
    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    keep, batches = _batches_for(specs, k32, k64)
    plan = pmp.Plan(0)
    say("case autotune")
    best = pmp.pmp_plan_autotune(plan, batches)
    say(f"best {best}")
    assert best["ms"] > 0 and best["alpha"] in (256, 512, 768, 1024, 1536, 2048)
    for rg, flags, buf, off, out in keep:
        out.zero_()
    pmp.pmp_hash_many(batches, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_OK
    for rg, flags, buf, off, out in keep:
        assert U.first_mismatch(U.as_u64(out.cpu().numpy()), oracle_of(rg, flags)) is None
    plan.close()


@pytest.mark.parametrize("shares", [2, 4, 16])
def test_shares_per_wave(shares):
    """Work spread over several shares per wave gives the same outputs."""
    import torch

    from paper_1609_09840_amd import pmp

    lens, wide = W.c4_lengths(6000, seed=951)
    specs = [(W.from_lengths(lens[~wide], 952, False), 0), (W.from_lengths(lens[wide], 953, True), 2)]
    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    keep, batches = _batches_for(specs, k32, k64)
    plan = pmp.Plan(0)
    plan.tune(0, 0, 1024, shares)
    say(f"case shares={shares}")
    pmp.pmp_hash_many(batches, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_OK
    for rg, flags, buf, off, out in keep:
        assert U.first_mismatch(U.as_u64(out.cpu().numpy()), oracle_of(rg, flags)) is None
    plan.close()


def test_graph_survives_workspace_growth():
    """A graph keeps using its workspace after a larger call on the same plan
    has grown the plan's workspace; its replays stay exact."""
    import torch

    from paper_1609_09840_amd import pmp

    rng = np.random.default_rng(970)
    small = [(W.from_lengths(rng.integers(0, 3000, size=300), 971, False), 0),
             (W.from_lengths(rng.integers(0, 3000, size=200), 972, True), 0)]
    big = [(W.from_lengths(rng.integers(0, 200000, size=3000), 973, False), 0)]
    k32 = U.to_dev_keys(U.keys_for(False, W.KEY_SEED32))
    k64 = U.to_dev_keys(U.keys_for(True, W.KEY_SEED64))
    keep_s, batches_s = _batches_for(small, k32, k64)
    keep_b, batches_b = _batches_for(big, k32, k64)
    plan = pmp.Plan(0)
    say("case graph growth")
    g = pmp.Graph(plan, batches_s)
    g.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    pmp.pmp_hash_many(batches_b, plan=plan)  # grows the workspace
    torch.cuda.synchronize()
    assert plan.status() == pmp.PMP_OK
    for rg, flags, buf, off, out in keep_b:
        assert U.first_mismatch(U.as_u64(out.cpu().numpy()), oracle_of(rg, flags)) is None
    for rep in range(2):
        for rg, flags, buf, off, out in keep_s:
            out.zero_()
        g.launch(torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert plan.status() == pmp.PMP_OK
        for rg, flags, buf, off, out in keep_s:
            assert U.first_mismatch(U.as_u64(out.cpu().numpy()), oracle_of(rg, flags)) is None, rep
    g.close()
    plan.close()
