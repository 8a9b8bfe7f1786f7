"""Serving through the C ABI (odp_server_*): every request's digest is the same
in the mix as alone and as the oracle's; the flags the server decided before
the drain equal the oracle's for every record whose deciding records had
arrived, and are unset for the others; the final flags after draining equal the
oracle's analysis of the arrival-ordered log. All bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

from gpu_helpers import compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F_DD, F_RT_TX, F_RT_RX, F_RA, F_UA, F_PAIRED, F_UT, F_INVALID = 1, 2, 4, 8, 16, 32, 64, 128
# decided once the whole log has arrived: at a record's arrival, or when a
# later record (a transfer back, a pairing) arrives
EXACT = F_DD | F_RT_TX | F_RT_RX | F_RA | F_PAIRED | F_INVALID


def decided_windows(ev, valid):
    """Which records' UA and UT bits the server has decided by the end of the
    log: a paired ALLOC whose DELETE ends before the last record starts; a copy
    into a device (H2D or D2D) whose next copy of the same (receiver, sender,
    source address) starts before the last record starts. Without a rejected
    record only (otherwise they wait for the drain)."""
    n = len(ev)
    ua = np.zeros(n, dtype=bool)
    ut = np.zeros(n, dtype=bool)
    if n == 0 or not valid.all():
        return ua, ut
    last = int(ev["t_start"][-1])
    open_ad = {}
    nxt = {}
    for i in range(n):
        op = int(ev["op"][i])
        if op in (1, 5):
            k = (int(ev["dst_dev"][i]), int(ev["dst_addr"][i]))
            if op == 5 and k in open_ad and int(ev["op"][open_ad[k]]) == 1 and int(ev["t_end"][i]) < last:
                ua[open_ad[k]] = True
            open_ad[k] = i
        elif op in (2, 4) and int(ev["dst_dev"][i]) >= 0:
            k = (int(ev["dst_dev"][i]), int(ev["src_dev"][i]), int(ev["src_addr"][i]))
            if k in nxt and int(ev["t_start"][i]) < last:
                ut[nxt[k]] = True
            nxt[k] = i
    return ua, ut


@pytest.fixture(scope="module")
def arena(odp):
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    a = torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device="cuda", generator=gen)
    return a, a.cpu().numpy()


def oracle_events(sched, host_arena):
    """The schedule's records with digests taken by the oracle from the payload bytes."""
    ev = sched.events.copy()
    cache = {}
    for i in np.nonzero(sched.payload_off >= 0)[0]:
        key = (int(sched.payload_off[i]), int(sched.payload_bytes[i]))
        if key not in cache:
            o, b = key
            cache[key] = oracle.d64(host_arena[o:o + b])
        ev["digest"][i] = cache[key]
    return ev


def served(odp, sched, **kw):
    srv = odp.Server(max_events=kw.pop("max_events", len(sched.events)), **kw)
    done, stats = srv.run(sched.events, sched.payload_ptrs(), sched.payload_bytes, sched.arrival_ns)
    log = srv.log().view(W.EVENT_DTYPE)
    imm, fl, rep = srv.drain()
    srv.close()
    return log, imm, fl, rep, done, stats


def check_served(odp, sched, ev_o, log, imm, fl, rep):
    tx = sched.payload_off >= 0
    assert (log["digest"][tx] == ev_o["digest"][tx]).all(), "served digests differ from the oracle"
    assert (log["digest"][~tx] == sched.events["digest"][~tx]).all()
    for f in ("src_addr", "dst_addr", "bytes", "t_start", "t_end", "op", "src_dev", "dst_dev"):
        assert (log[f] == sched.events[f]).all(), f
    fo, ro = oracle.analyze(ev_o)
    compare(fl, rep, fo, ro)
    check_known(imm, fo, ev_o)
    return fo, ro


def check_known(known, fo, ev):
    bad = np.nonzero((known & EXACT) != (fo & EXACT))[0]
    assert bad.size == 0, "flags decided before the drain differ at %s: %s vs %s" % (
        bad[:10].tolist(), known[bad[:10]].tolist(), fo[bad[:10]].tolist())
    valid = (fo & F_INVALID) == 0
    ua, ut = decided_windows(ev, valid)
    for bit, dec in ((F_UA, ua), (F_UT, ut)):
        if valid.all():
            want = np.where(dec, fo & bit, 0)
            diff = np.nonzero((known & bit) != want)[0]
            assert diff.size == 0, "bit %d before the drain differs at %s" % (bit, diff[:10].tolist())
    return ua, ut


@pytest.mark.parametrize("max_tick", [1, 7, 1024])
def test_serve_mix_equals_alone_and_oracle(odp, arena, max_tick):
    a, host = arena
    sched = W.ServingSchedule(seed=21, n=2500, rate=50_000.0, lo=4096, hi=1 << 20, arena=a)
    ev_o = oracle_events(sched, host)
    log, imm, fl, rep, done, stats = served(odp, sched, budget_bytes=256 << 20, max_tick=max_tick)
    fo, ro = check_served(odp, sched, ev_o, log, imm, fl, rep)
    assert ro["dd_events"] > 100 and ro["rt_rx_events"] > 10 and ro["n_alloc_pairs"] > 10
    assert stats["max_tick"] <= max_tick and stats["bytes"] == int(sched.payload_bytes.sum())
    assert (done >= sched.arrival_ns).all()
    # alone: each sampled request digested by itself, in its own call
    rng = np.random.default_rng(3)
    idx = rng.choice(np.nonzero(sched.payload_off >= 0)[0], size=120, replace=False)
    for i in idx:
        o, b = int(sched.payload_off[i]), int(sched.payload_bytes[i])
        alone = odp.digest_tensors([a[o:o + b]])[0]
        assert alone == log["digest"][i], "request %d: alone %x, in the mix %x" % (i, alone, log["digest"][i])


def test_serve_burst_over_budget(odp, arena):
    """All requests at t = 0, four payloads' worth of budget: admission waits,
    ticks stay within the budget, results unchanged."""
    a, host = arena
    sched = W.ServingSchedule(seed=22, n=96, rate=1e6, lo=4 << 20, hi=4 << 20, arena=a)
    sched.arrival_ns[:] = 0
    ev_o = oracle_events(sched, host)
    log, imm, fl, rep, done, stats = served(odp, sched, budget_bytes=16 << 20)
    check_served(odp, sched, ev_o, log, imm, fl, rep)
    assert stats["budget_waits"] > 0
    assert stats["bytes"] == int(sched.payload_bytes.sum())


def test_serve_slots_and_plain_mode(odp, arena):
    """A slot limit and the plain mode (one request per launch) give the batched results."""
    a, host = arena
    sched = W.ServingSchedule(seed=23, n=600, rate=1e6, lo=4096, hi=256 << 10, arena=a)
    ev_o = oracle_events(sched, host)
    r_slots = served(odp, sched, budget_bytes=64 << 20, max_inflight=5)
    check_served(odp, sched, ev_o, *r_slots[:4])
    assert r_slots[5]["max_tick"] <= 5
    r_plain = served(odp, sched, budget_bytes=64 << 20, mode=odp.SERVER_PLAIN)
    check_served(odp, sched, ev_o, *r_plain[:4])
    assert r_plain[5]["ticks"] == len(sched.events)


def test_serve_runs_append_and_invalid_records(odp, arena):
    """Two runs on one server form one log; records that break the log's
    order or carry bad devices are INVALID at arrival and after draining."""
    a, host = arena
    s1 = W.ServingSchedule(seed=24, n=700, rate=200_000.0, lo=4096, hi=64 << 10, arena=a)
    s2 = W.ServingSchedule(seed=25, n=500, rate=200_000.0, lo=4096, hi=64 << 10, arena=a)
    s2.events["t_start"] += s1.events["t_start"][-1]
    s2.events["t_end"] += s1.events["t_start"][-1]
    rng = np.random.default_rng(5)
    for k in rng.choice(np.arange(1, 500), size=12, replace=False):
        s2.events["t_start"][k] = s2.events["t_start"][k - 1] - 1 if s2.events["t_start"][k - 1] else 0
    s2.events["dst_dev"][[3, 40]] = 12
    srv = odp.Server(max_events=1200, budget_bytes=64 << 20, max_tick=64)
    srv.run(s1.events, s1.payload_ptrs(), s1.payload_bytes, s1.arrival_ns)
    srv.run(s2.events, s2.payload_ptrs(), s2.payload_bytes, s2.arrival_ns)
    log = srv.log().view(W.EVENT_DTYPE)
    imm, fl, rep = srv.drain()
    with pytest.raises(odp.OdpError):
        srv.run(s1.events[:1], s1.payload_ptrs()[:1], s1.payload_bytes[:1], s1.arrival_ns[:1])
    srv.close()
    ev_o = np.concatenate([oracle_events(s1, host), oracle_events(s2, host)])
    both = W.ServingSchedule.__new__(W.ServingSchedule)
    both.events = np.concatenate([s1.events, s2.events])
    both.payload_off = np.concatenate([s1.payload_off, s2.payload_off])
    fo, ro = check_served(odp, both, ev_o, log, imm, fl, rep)
    assert ro["n_invalid"] >= 12 and ro["status"] == 1


def test_serve_rejects_bad_requests(odp):
    ev = W.empty_events(3)
    ev["op"] = W.H2D
    ev["src_dev"], ev["dst_dev"] = W.HOST, 0
    buf = torch.zeros(8 << 20, dtype=torch.uint8, device="cuda")
    ptrs = np.full(3, buf.data_ptr(), dtype=np.uint64)
    srv = odp.Server(max_events=8, budget_bytes=1 << 20)
    with pytest.raises(odp.OdpError) as e:
        srv.run(ev, ptrs, np.array([16, 2 << 20, 16], dtype=np.uint64), np.zeros(3, dtype=np.uint64))
    assert e.value.code == odp.ODP_EINVAL
    with pytest.raises(odp.OdpError) as e:
        srv.run(ev, ptrs, np.full(3, 16, dtype=np.uint64), np.array([5, 4, 6], dtype=np.uint64))
    assert e.value.code == odp.ODP_EINVAL
    with pytest.raises(odp.OdpError) as e:
        srv.run(ev, np.zeros(3, dtype=np.uint64), np.full(3, 16, dtype=np.uint64), np.zeros(3, dtype=np.uint64))
    assert e.value.code == odp.ODP_EINVAL
    srv.close()
    with pytest.raises(odp.OdpError):
        odp.Server(max_events=8, budget_bytes=1 << 20, max_tick=2000)
    with pytest.raises(odp.OdpError):
        odp.Server(max_events=0, budget_bytes=1 << 20)


def test_servers_release_their_memory(odp, arena):
    """Creating, running, draining and destroying servers in a loop leaves the
    device's free memory where it was after the first cycle: a server frees
    its own buffers and the workspace the library kept for its stream."""
    a, host = arena
    sched = W.ServingSchedule(seed=26, n=20_000, rate=2e6, lo=4096, hi=64 << 10, arena=a)

    def cycle():
        srv = odp.Server(max_events=len(sched.events), budget_bytes=1 << 30)
        srv.run(sched.events, sched.payload_ptrs(), sched.payload_bytes, sched.arrival_ns)
        srv.drain()
        srv.close()
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    first = cycle()
    for _ in range(6):
        last = cycle()
    # one cycle's workspace alone is several MiB (the drain's analysis of
    # 20,000 records and the digest reserve); a leak would accumulate six
    assert abs(int(first) - int(last)) < (4 << 20), (first, last)


@pytest.mark.parametrize("max_tick", [1, 5, 1024])
def test_flags_decided_before_the_drain(odp, arena, max_tick):
    """Round trips sent back several ticks later, repeated and unused
    allocations, copies overwritten before any kernel: every bit a record can
    have is set before the drain once its deciding records have arrived, equal
    to the oracle's, in ticks of one record, of a few and of many."""
    a, host = arena
    sched = W.ServingSchedule(seed=27, n=4000, rate=100_000.0, lo=4096, hi=256 << 10, arena=a)
    ev_o = oracle_events(sched, host)
    log, imm, fl, rep, done, stats = served(odp, sched, budget_bytes=512 << 20, max_tick=max_tick)
    fo, ro = check_served(odp, sched, ev_o, log, imm, fl, rep)
    ua, ut = decided_windows(ev_o, (fo & F_INVALID) == 0)
    for bit, name in ((F_RT_TX, "rt_pairs"), (F_RA, "ra_events")):
        assert int(((imm & bit) != 0).sum()) == ro[name] > 0
    assert ((imm & F_UA) != 0).sum() > 0 and ((imm & F_UT) != 0).sum() > 0
    assert ua.sum() > 0.9 * ((fo & F_PAIRED) != 0).sum() / 2  # nearly every window closed by the end
