"""GPU parity of the trace analysis against the CPU oracle: every flag and
every report field bit-exact, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

from golden_traces import load as load_golden
from gpu_helpers import analyze_gpu, compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def with_digests(ev, payloads, payload_of):
    ev = ev.copy()
    dg = [oracle.d64(p) for p in payloads]
    for i in range(len(ev)):
        if payload_of[i] >= 0:
            ev["digest"][i] = dg[payload_of[i]]
    return ev


def check(odp, ev):
    fr, rr = oracle.analyze(ev)
    fg, rg = analyze_gpu(odp, ev)
    compare(fg, rg, fr, rr)
    return fg, rg


def test_empty_log(odp):
    fg, rg = analyze_gpu(odp, W.empty_events(0))
    assert rg["n_events"] == 0 and rg["status"] == 0 and rg["first_bad_event"] == 0xFFFFFFFF


@pytest.mark.parametrize("name", ["listing1_trace.txt", "listing2_trace.txt"])
def test_paper_listings(odp, name):
    ev, payloads, payload_of, expect = load_golden(name)
    fg, rg = check(odp, with_digests(ev, payloads, payload_of))
    for k, v in expect.items():
        assert rg[k] == v, k


def test_tiny_random_traces(odp):
    for seed in range(400):
        n_dev = 1 + seed % 3
        inv = 0.1 if seed % 4 == 0 else 0.0
        ev, payloads, payload_of = W.tiny_trace(seed, n_events=1 + (seed * 7) % 90, n_devices=n_dev,
                                                 invalid_rate=inv, overlap_kernels=seed % 5 == 0)
        check(odp, with_digests(ev, payloads, payload_of))


def test_traces_spanning_many_tiles(odp):
    """Digest groups and ALLOC/DELETE groups that cross 4,096-record tiles."""
    for seed, n in [(1, 5000), (2, 12289), (3, 40000)]:
        ev, payloads, payload_of = W.tiny_trace(1000 + seed, n_events=n, n_devices=3, n_payloads=5, n_vars=3,
                                                 invalid_rate=0.01)
        check(odp, with_digests(ev, payloads, payload_of))


def test_one_giant_group(odp):
    """Every record carries the same digest: one group spanning every tile."""
    m = 50_000
    ev = W.empty_events(m)
    rng = np.random.default_rng(5)
    src = rng.integers(-1, 3, size=m)
    dst = rng.integers(-1, 3, size=m)
    ev["op"] = W.D2D
    ev["src_dev"], ev["dst_dev"] = src, dst
    ev["digest"] = 0x1234
    ev["t_start"] = np.arange(m) * 10
    ev["t_end"] = ev["t_start"] + 5
    check(odp, ev)


def test_all_endpoints_and_self_transfers(odp):
    rng = np.random.default_rng(6)
    m = 20_000
    ev = W.empty_events(m)
    ev["op"] = rng.choice([W.H2D, W.D2H, W.D2D], size=m)
    ev["src_dev"] = rng.integers(-1, 10, size=m)
    ev["dst_dev"] = rng.integers(-1, 10, size=m)
    ev["digest"] = rng.integers(0, 40, size=m).astype(np.uint64)
    ev["t_start"] = np.arange(m)
    ev["t_end"] = ev["t_start"]
    check(odp, ev)


def test_sentinel_digest_and_ties(odp):
    """A transfer whose digest is all ones sorts among the non-transfer records;
    equal timestamps keep array order."""
    ev = W.empty_events(8)
    ev["op"] = [W.ALLOC, W.H2D, W.KERNEL, W.H2D, W.D2H, W.H2D, W.DELETE, W.H2D]
    ev["src_dev"] = [-1, -1, -1, -1, 0, -1, -1, -1]
    ev["dst_dev"] = [0, 0, 0, 0, -1, 0, 0, 0]
    ev["digest"] = [0, 2**64 - 1, 0, 2**64 - 1, 2**64 - 1, 7, 0, 2**64 - 1]
    ev["t_start"] = [0, 0, 0, 1, 1, 1, 2, 2]
    ev["t_end"] = ev["t_start"] + 1
    check(odp, ev)


def test_invalid_records(odp):
    for seed in range(30):
        ev, payloads, payload_of = W.tiny_trace(5000 + seed, n_events=300, n_devices=2, invalid_rate=0.3)
        fg, rg = check(odp, with_digests(ev, payloads, payload_of))
        assert rg["status"] in (0, 1)


def test_plain_small_end_to_end(odp):
    """Digests of every snapshot on the GPU (per-buffer launches), then the
    analysis on the GPU; the oracle digests and analyses the same bytes."""
    ps = W.PlainSmall(seed=1)
    snaps = [torch.from_numpy(s).to("cuda") for s in ps.snapshots]
    gd = odp.digest_tensors(snaps, plain=True)
    od = np.array([oracle.d64(s) for s in ps.snapshots], dtype=np.uint64)
    assert (gd == od).all()
    ev_g = ps.events.copy()
    ev_o = ps.events.copy()
    m = ps.snapshot_of >= 0
    ev_g["digest"][m] = gd[ps.snapshot_of[m]]
    ev_o["digest"][m] = od[ps.snapshot_of[m]]
    fr, rr = oracle.analyze(ev_o)
    fg, rg = analyze_gpu(odp, ev_g)
    compare(fg, rg, fr, rr)
    assert all(fg[i] & odp.F_DD for i in ps.planted_dd)
    assert all(fg[i] & odp.F_RT_RX for i in ps.planted_rt_rx)


def test_trace_at_scale_full_size(odp):
    """10^7 map records over 10^5 Zipf(1.1) slots plus kernel records: every flag
    against the oracle, and the planted counts exactly."""
    tr = W.TraceAtScale(seed=4)
    fg, rg = analyze_gpu(odp, tr.events)
    for k, v in tr.planted.items():
        assert rg[k] == v, k
    fr, rr = oracle.analyze(tr.events)
    compare(fg, rg, fr, rr)


def test_repeated_calls_and_streams(odp):
    ev, payloads, payload_of = W.tiny_trace(77, n_events=3000, n_devices=3, n_payloads=4)
    ev = with_digests(ev, payloads, payload_of)
    fr, rr = oracle.analyze(ev)
    for _ in range(3):
        fg, rg = analyze_gpu(odp, ev)
        compare(fg, rg, fr, rr)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fg, rg = analyze_gpu(odp, ev, stream=s)
    compare(fg, rg, fr, rr)
    # a smaller log after a larger one reuses the workspace
    small = ev[:100].copy()
    fr2, rr2 = oracle.analyze(small)
    fg2, rg2 = analyze_gpu(odp, small)
    compare(fg2, rg2, fr2, rr2)


def test_null_report_rejected(odp):
    import ctypes
    rc = odp.load().odp_analyze_trace(None, 0, None, None, None)
    assert rc == odp.ODP_EINVAL


def test_analysis_replayed_from_a_graph(odp):
    """A captured analysis (its side-stream fork and join included) replays
    correctly several times, with eager work on the buffers between replays."""
    tr = W.TraceAtScale(seed=9, n_map=200_000, n_slots=5_000)
    ev = tr.events
    n = len(ev)
    fr, rr = oracle.analyze(ev)
    s = torch.cuda.Stream()
    d_ev = torch.from_numpy(ev.view(np.uint8).reshape(-1).copy()).to("cuda")
    d_flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        odp.reserve(max_events=n, stream=s)
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=s, n=n)
    s.synchronize()
    compare(d_flags.cpu().numpy(), odp.report_to_dict(d_rep.cpu().numpy()), fr, rr)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=s, n=n)
    for _ in range(3):
        d_flags.fill_(0xAA)
        d_rep.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        compare(d_flags.cpu().numpy(), odp.report_to_dict(d_rep.cpu().numpy()), fr, rr)


@pytest.mark.parametrize("n", [1, 511, 512, 513, 2047, 2048, 2049, 4200])
def test_one_workgroup_sort_threshold(odp, n):
    """Logs of at most 512 records are analysed by one workgroup (each rule
    written out per record), up to 2,048 records take the one-workgroup sorts,
    longer ones the multi-launch passes; every side of both thresholds matches
    the oracle (three devices, rejected records, multi-word keys)."""
    ev, payloads, payload_of = W.tiny_trace(300 + n, n_events=n, n_devices=3, n_payloads=6, invalid_rate=0.01)
    ev = with_digests(ev, payloads, payload_of)
    check(odp, ev)
    clean, payloads, payload_of = W.tiny_trace(400 + n, n_events=n, n_devices=2, n_payloads=6)
    check(odp, with_digests(clean, payloads, payload_of))


@pytest.mark.parametrize("m,seed", [(30_000, 1), (1_000_000, 2)])
def test_digests_sharing_low_bytes(odp, m, seed):
    """The digest sort first orders by the low bytes only (3 of them at 30,000
    records and at a million, 4 at ten million); runs of equal low bytes that hold several digests
    are then sorted in place by the whole digest when they are short, and
    switch every remaining pass on when one is long. Planted digests that differ
    from another only in byte 6 or 7, or only in byte 4, interleaved in time
    with it, land in short mixed runs (else their groups interleave and the
    flags go wrong); unrelated random digests take whatever the checks find.
    Every case must give the oracle's result."""
    rng = np.random.default_rng(seed)
    ev = W.empty_events(m)
    ev["op"] = rng.choice([W.H2D, W.D2H, W.D2D], size=m)
    ev["src_dev"] = rng.integers(-1, 3, size=m)
    ev["dst_dev"] = rng.integers(-1, 3, size=m)
    ev["t_start"] = np.arange(m, dtype=np.uint64) * 3
    ev["t_end"] = ev["t_start"] + 2
    top = np.uint64(0xFFFFFFFFFFFFFFFE)
    base = rng.integers(0, top, size=m // 4, dtype=np.uint64, endpoint=True)
    dig = rng.choice(base, size=m)
    flip = rng.random(m) < 0.2
    which = rng.integers(0, 2, size=m)
    high = np.where(flip & (which == 0), dig ^ np.uint64(0x5A << 56), dig)
    high = np.where(flip & (which == 1), high ^ np.uint64(1 << 48), high)
    for digests in (high, np.where(flip, dig ^ np.uint64(1 << 32), dig),
                    rng.integers(0, top, size=m, dtype=np.uint64, endpoint=True)):
        ev["digest"] = digests
        fg, rg = check(odp, ev)
    ev["digest"] = high
    fg, rg = check(odp, ev)
    assert rg["dd_events"] > m // 4 and rg["rt_pairs"] > 0


@pytest.mark.parametrize("m,byte", [(30_000, 7), (30_000, 3), (1_000_000, 5)])
def test_long_runs_of_shared_low_bytes(odp, m, byte):
    """Two groups of 400 records each whose digests differ only in one high
    byte, interleaved in time, form one run of equal low bytes longer than any
    run sorted in place (in the low 3 or 4 bytes the first passes sort, or in
    a higher byte): the remaining passes must run, and the other records
    (random digests, some in short mixed runs) still come out right."""
    rng = np.random.default_rng(m + byte)
    ev = W.empty_events(m)
    ev["op"] = rng.choice([W.H2D, W.D2H, W.D2D], size=m)
    ev["src_dev"] = rng.integers(-1, 3, size=m)
    ev["dst_dev"] = rng.integers(-1, 3, size=m)
    ev["t_start"] = np.arange(m, dtype=np.uint64) * 3
    ev["t_end"] = ev["t_start"] + 2
    top = np.uint64(0xFFFFFFFFFFFFFFFE)
    base = rng.integers(0, top, size=m // 8, dtype=np.uint64, endpoint=True)
    dig = rng.choice(base, size=m)
    dig = np.where(rng.random(m) < 0.1, dig ^ np.uint64(1 << 60), dig)
    a = np.uint64(0x0123456789ABCDEF)
    pos = rng.choice(m, size=800, replace=False)
    dig[pos[:400]] = a
    dig[pos[400:]] = a ^ np.uint64(0x80 << (8 * byte))
    ev["digest"] = dig
    fg, rg = check(odp, ev)
    assert rg["dd_events"] >= 792


def big_subset_log(rng, m, kind):
    """m records, nearly all KERNELs (kind "kernel") or nearly all ALLOC/DELETE
    records (kind "alloc"), over host + 3 devices, with some transfers: each
    of the allocation-path sorts then has more than 512 tiles of 4,096."""
    ev = W.empty_events(m)
    t = np.cumsum(rng.integers(0, 3, size=m)).astype(np.uint64)
    ev["t_start"] = t
    ev["t_end"] = t + rng.integers(0, 3, size=m).astype(np.uint64)
    dev = rng.integers(0, 3, size=m)
    if kind == "kernel":
        op = np.where(rng.random(m) < 0.96, W.KERNEL, 0)
        op = np.where((op == 0) & (rng.random(m) < 0.5), W.ALLOC, op)
        op = np.where(op == 0, W.DELETE, op)
    else:
        op = np.where(rng.random(m) < 0.5, W.ALLOC, W.DELETE)
        op = np.where(rng.random(m) < 0.03, W.KERNEL, op)
    tx = rng.random(m) < 0.01
    op = np.where(tx, W.H2D, op)
    ev["op"] = op
    ev["src_dev"] = np.where(tx, W.HOST, W.HOST)
    ev["dst_dev"] = dev
    var = rng.integers(0, 5000, size=m).astype(np.uint64)
    ev["src_addr"] = np.uint64(W.HOST_BASE) + var * np.uint64(4096)
    ev["dst_addr"] = np.uint64(W.DEV_BASE) + var * np.uint64(4096)
    ev["bytes"] = np.where(op == W.KERNEL, 0, rng.choice([64, 128, 4096], size=m)).astype(np.uint64)
    ev["digest"] = np.where(tx, rng.integers(0, 1 << 20, size=m).astype(np.uint64), np.uint64(0))
    return ev


@pytest.mark.parametrize("kind", ["kernel", "alloc"])
def test_allocation_path_sorts_loop_over_tiles(odp, kind):
    """The allocation-path sorts run a capped number of blocks per job (twice
    the compute units) that loop over the job's tiles; logs whose KERNEL or
    ALLOC/DELETE subset spans more tiles than that must match the oracle."""
    ev = big_subset_log(np.random.default_rng(31 if kind == "kernel" else 32), 2_400_000, kind)
    fg, rg = check(odp, ev)
    if kind == "kernel":
        assert rg["n_kernels"] > 2_100_000
    else:
        assert rg["n_alloc_pairs"] > 100_000 and rg["ra_events"] > 0


def test_log_above_packed_index_limit(odp):
    """Logs of fewer than 2^24 records carry the endpoint code in the top byte
    of the digest sort's values; a longer log keeps plain indices and gathers
    the codes. 2^24 + 70,000 records of transfers (repeated digests, three
    devices), kernels and ALLOC/DELETE records must match the oracle."""
    m = (1 << 24) + 70_000
    rng = np.random.default_rng(33)
    ev = W.empty_events(m)
    t = np.cumsum(rng.integers(0, 3, size=m)).astype(np.uint64)
    ev["t_start"] = t
    ev["t_end"] = t + 1
    op = rng.choice([W.H2D, W.D2H, W.D2D, W.KERNEL, W.ALLOC, W.DELETE], size=m,
                    p=[0.4, 0.3, 0.1, 0.1, 0.05, 0.05])
    ev["op"] = op
    src = rng.integers(-1, 3, size=m)
    dst = rng.integers(-1, 3, size=m)
    src = np.where(op == W.H2D, -1, np.where(op == W.D2H, np.maximum(src, 0), np.maximum(src, 0)))
    dst = np.where(op == W.D2H, -1, np.maximum(dst, 0))
    ev["src_dev"], ev["dst_dev"] = src, dst
    pool = rng.integers(0, np.uint64(0xFFFFFFFFFFFFFFFE), size=m // 3, dtype=np.uint64, endpoint=True)
    is_tx = np.isin(op, [W.H2D, W.D2H, W.D2D])
    ev["digest"] = np.where(is_tx, rng.choice(pool, size=m), np.uint64(0))
    var = rng.integers(0, 20_000, size=m).astype(np.uint64)
    ev["src_addr"] = np.uint64(W.HOST_BASE) + var * np.uint64(4096)
    ev["dst_addr"] = np.uint64(W.DEV_BASE) + var * np.uint64(4096)
    ev["bytes"] = np.where(op == W.KERNEL, 0, 4096).astype(np.uint64)
    fg, rg = check(odp, ev)
    assert rg["n_events"] == m and rg["dd_events"] > 1_000_000 and rg["rt_pairs"] > 1000


@pytest.mark.parametrize("pairs,keys,hot", [(1000, 500, 0.0), (150_000, 100_000, 0.5), (40_000, 3, 0.0)])
def test_allocation_groups_of_every_size(odp, pairs, keys, hot):
    """Paired allocations grouped by (host address, device, bytes) for RA: a
    table barely larger than the keys (many probes run into each other), one
    key holding half of 150,000 pairs (many lanes of a wavefront share it),
    and three keys for 40,000 pairs; each against the oracle."""
    rng = np.random.default_rng(pairs + keys)
    m = 2 * pairs
    ev = W.empty_events(m)
    ev["op"] = np.tile([W.ALLOC, W.DELETE], pairs)
    key = rng.integers(0, keys, size=pairs)
    key = np.where(rng.random(pairs) < hot, 0, key)
    dev = (key % 3).astype(np.int8)
    ev["dst_dev"] = np.repeat(dev, 2)
    ev["src_dev"] = -1
    ev["src_addr"] = np.repeat(np.uint64(W.HOST_BASE) + (key // 3).astype(np.uint64) * np.uint64(4096), 2)
    ev["bytes"] = np.repeat(np.uint64(64) << (key % 5).astype(np.uint64), 2)
    ev["dst_addr"] = np.repeat(np.uint64(W.DEV_BASE) + np.arange(pairs, dtype=np.uint64) * np.uint64(64), 2)
    ev["t_start"] = np.arange(m, dtype=np.uint64) * 2
    ev["t_end"] = ev["t_start"] + 1
    kern = rng.random(m) < 0.02
    ev["op"] = np.where(kern, W.KERNEL, ev["op"])
    ev["bytes"] = np.where(kern, 0, ev["bytes"])
    fg, rg = check(odp, ev)
    assert rg["ra_events"] > 0


@pytest.mark.parametrize("m,tx_share", [(5_000, 0.5), (20_000, 0.02), (20_000, 0.0), (3_000, 1.0)])
def test_digest_sort_keeps_only_transfers(odp, m, tx_share):
    """The digest sort's first pass drops every record that is not a valid
    transfer (KERNEL, ALLOC/DELETE, rejected records), which carry the
    all-ones sort key. Transfers whose digest is itself all ones, or shares
    its low bytes with it, must still be grouped with each other and nothing
    else: logs from no transfers at all to transfers only, with rejected
    records sprinkled in, must match the oracle."""
    rng = np.random.default_rng(int(m * 10 + tx_share * 100))
    ev = W.empty_events(m)
    t = np.cumsum(rng.integers(0, 3, size=m)).astype(np.uint64)
    ev["t_start"] = t
    ev["t_end"] = t + 1
    is_tx = rng.random(m) < tx_share
    ev["op"] = np.where(is_tx, rng.choice([W.H2D, W.D2H, W.D2D], size=m),
                        rng.choice([W.KERNEL, W.ALLOC, W.DELETE], size=m))
    op = ev["op"]
    src = rng.integers(0, 3, size=m)
    dst = rng.integers(0, 3, size=m)
    ev["src_dev"] = np.where(op == W.H2D, -1, src)
    ev["dst_dev"] = np.where(op == W.D2H, -1, dst)
    ones = np.uint64(0xFFFFFFFFFFFFFFFF)
    pool = np.array([ones, ones ^ np.uint64(1 << 63), ones ^ np.uint64(1 << 40), 7, 8], dtype=np.uint64)
    ev["digest"] = np.where(is_tx, rng.choice(pool, size=m), rng.integers(0, 1 << 62, size=m).astype(np.uint64))
    var = rng.integers(0, 50, size=m).astype(np.uint64)
    ev["src_addr"] = np.uint64(W.HOST_BASE) + var * np.uint64(4096)
    ev["dst_addr"] = np.uint64(W.DEV_BASE) + var * np.uint64(4096)
    ev["bytes"] = np.uint64(4096)
    bad = rng.random(m) < 0.01
    ev["t_end"][bad] = ev["t_start"][bad] - np.uint64(1) * (ev["t_start"][bad] > 0)
    ev["dst_dev"][bad & (ev["t_start"] == 0)] = 42
    check(odp, ev)
