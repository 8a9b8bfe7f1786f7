"""Pins of the oracle's detection rules against things other than itself:
brute force over the paper's definitions with byte equality (tests/brute.py,
every flag and every count and sum of the report), the worked examples of the
paper's Listings 1 and 2 (tests/golden/), closed forms, the planted counts and
sums of the synthetic generators, and the pairs Algorithm 2 records.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2601_12713_amd import workloads as W

from brute import brute
from golden_traces import load as load_golden


def with_digests(ev, payloads, payload_of):
    ev = ev.copy()
    dg = [oracle.d64(p) for p in payloads]
    for i in range(len(ev)):
        if payload_of[i] >= 0:
            ev["digest"][i] = dg[payload_of[i]]
    return ev


def check_against_brute(ev, payloads, payload_of):
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    bflags, bc = brute(ev, lambda i: payloads[payload_of[i]])
    assert flags.tolist() == bflags
    for k, v in bc.items():
        assert rep[k] == v, (k, rep[k], v)
    return flags, rep


@settings(max_examples=250, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n_dev=st.integers(1, 3), n=st.integers(0, 60))
def test_rules_match_brute_force(seed, n_dev, n):
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=n, n_devices=n_dev, n_payloads=6, n_vars=3)
    check_against_brute(ev, payloads, payload_of)


@settings(max_examples=150, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n=st.integers(1, 60))
def test_rules_match_brute_force_with_invalid_records(seed, n):
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=n, n_devices=2, invalid_rate=0.15)
    flags, rep = check_against_brute(ev, payloads, payload_of)
    bad = np.nonzero(flags & oracle.F_INVALID)[0]
    if bad.size:
        assert rep["status"] == 1 and rep["first_bad_event"] == int(bad[0])
    else:
        assert rep["status"] == 0 and rep["first_bad_event"] == 0xFFFFFFFF


@settings(max_examples=100, deadline=None)
@given(seed=st.integers(0, 2**32 - 1))
def test_rules_match_brute_force_overlapping_kernels(seed):
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=50, n_devices=2, overlap_kernels=True)
    check_against_brute(ev, payloads, payload_of)


def test_report_sums_of_bytes_and_time():
    ev, payloads, payload_of = W.tiny_trace(4242, n_events=200, n_devices=2, n_payloads=5)
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    dur = (evd["t_end"] - evd["t_start"]).astype(np.int64)
    by = evd["bytes"].astype(np.int64)
    m = (flags & oracle.F_DD) != 0
    assert rep["dd_bytes"] == int(by[m].sum()) and rep["dd_time_ns"] == int(dur[m].sum())
    m = (flags & oracle.F_RT_RX) != 0
    assert rep["rt_bytes"] == int(by[m].sum()) and rep["rt_time_ns"] == int(dur[m].sum())
    assert rep["dd_members"] == rep["dd_events"] + rep["dd_groups"]
    assert rep["ra_members"] == rep["ra_events"] + rep["ra_groups"]


@pytest.mark.parametrize("name", ["listing1_trace.txt", "listing2_trace.txt"])
def test_paper_listings(name):
    ev, payloads, payload_of, expect = load_golden(name)
    flags, rep = check_against_brute(ev, payloads, payload_of)
    for k, v in expect.items():
        assert rep[k] == v, (k, rep[k], v)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 8, 11, 16])
def test_alternating_chain_closed_form(m):
    """m transfers of one content alternating host->dev0 / dev0->host: every
    send but the last has a later return, every record but the first is a
    return leg, and each side receives it ceil/floor(m/2) times."""
    ev = W.empty_events(m)
    for i in range(m):
        ev["op"][i] = W.H2D if i % 2 == 0 else W.D2H
        ev["src_dev"][i], ev["dst_dev"][i] = (-1, 0) if i % 2 == 0 else (0, -1)
        ev["t_start"][i], ev["t_end"][i] = 10 * i, 10 * i + 5
        ev["digest"][i] = 0xABCDEF
        ev["bytes"][i] = 8
    flags, rep = oracle.analyze(ev)
    assert rep["rt_pairs"] == m - 1
    assert rep["rt_rx_events"] == m - 1
    dev_rx, host_rx = (m + 1) // 2, m // 2
    assert rep["dd_events"] == max(dev_rx - 1, 0) + max(host_rx - 1, 0)
    if m % 2 == 0:
        assert rep["dd_events"] == m - 2


def _valid_transfers(ev, flags):
    return np.nonzero(((ev["op"] == W.H2D) | (ev["op"] == W.D2H) | (ev["op"] == W.D2D)) & ((flags & oracle.F_INVALID) == 0))[0]


@settings(max_examples=300, deadline=None)
@given(seed=st.integers(0, 2**32 - 1))
def test_algorithm2_matches_round_trip_rule_on_two_endpoints(seed):
    """With two endpoints per content, the <tx, rx> pairs Algorithm 2 records
    are exactly the RT_TX records, each paired with the first later reversed
    record, and the rx records are exactly the RT_RX records (the argument is
    written out with reading 4)."""
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=60, n_devices=1, n_payloads=4)
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    T = [i for i in _valid_transfers(evd, flags) if evd["src_dev"][i] != evd["dst_dev"][i]]
    pairs = oracle.alg2_pairs(evd, np.array(T, dtype=np.uint64))
    txs = sorted(T[t] for t, _ in pairs)
    assert txs == [i for i in T if flags[i] & oracle.F_RT_TX]
    assert len(pairs) == rep["rt_pairs"]
    for t, r in pairs:
        i, j = T[t], T[r]
        later = [k for k in T if k > i and evd["digest"][k] == evd["digest"][i]
                 and evd["src_dev"][k] == evd["dst_dev"][i] and evd["dst_dev"][k] == evd["src_dev"][i]]
        assert j == later[0]
    assert sorted({T[r] for _, r in pairs}) == [i for i in T if flags[i] & oracle.F_RT_RX]


def test_algorithm2_differs_with_three_endpoints():
    """The reading taken for three or more endpoints: Algorithm 2 can record a
    return leg that precedes the send and comes from a third device."""
    ev = W.empty_events(2)
    # dev1 -> host (h), then host -> dev0 (h)
    ev["op"] = [W.D2H, W.H2D]
    ev["src_dev"], ev["dst_dev"] = [1, -1], [-1, 0]
    ev["t_start"], ev["t_end"] = [0, 10], [5, 15]
    ev["digest"] = 77
    flags, rep = oracle.analyze(ev)
    assert rep["rt_pairs"] == 0
    pairs = oracle.alg2_pairs(ev, np.array([0, 1], dtype=np.uint64))
    assert pairs == [(1, 0)]


def test_no_kernels_means_every_pair_unused():
    ev = W.empty_events(4)
    ev["op"] = [W.ALLOC, W.DELETE, W.ALLOC, W.DELETE]
    ev["dst_dev"] = 0
    ev["src_dev"] = -1
    ev["dst_addr"] = W.DEV_BASE
    ev["src_addr"] = W.HOST_BASE
    ev["bytes"] = 64
    ev["t_start"], ev["t_end"] = [0, 10, 20, 30], [5, 15, 25, 35]
    flags, rep = oracle.analyze(ev)
    assert rep["ua_events"] == 2 and rep["ra_events"] == 1 and rep["n_alloc_pairs"] == 2


def test_kernel_touching_the_lifetime_counts_as_use():
    """Closed intervals: a kernel ending exactly when the allocation starts, or
    starting exactly when the deletion ends, meets the lifetime."""
    for ks, ke in [(0, 10), (40, 50)]:
        ev = W.empty_events(3)
        ev["op"] = [W.KERNEL, W.ALLOC, W.DELETE] if ks == 0 else [W.ALLOC, W.DELETE, W.KERNEL]
        ev["dst_dev"] = 0
        ev["src_dev"] = -1
        if ks == 0:
            ev["t_start"], ev["t_end"] = [ks, 10, 30], [ke, 20, 40]
        else:
            ev["t_start"], ev["t_end"] = [10, 30, ks], [20, 40, ke]
        flags, rep = oracle.analyze(ev)
        assert rep["n_alloc_pairs"] == 1 and rep["ua_events"] == 0


def test_empty_log():
    flags, rep = oracle.analyze(W.empty_events(0))
    assert flags.size == 0 and rep["n_events"] == 0 and rep["status"] == 0


def test_trace_at_scale_planted_counts_exact():
    tr = W.TraceAtScale(seed=4, n_map=300_000, n_slots=20_000)
    flags, rep = oracle.analyze(tr.events)
    for k, v in tr.planted.items():
        assert rep[k] == v, (k, rep[k], v)
    assert rep["status"] == 0
    assert rep["ut_events"] > 0 and rep["ra_bytes"] > 0 and rep["ua_time_ns"] > 0


def test_savings_estimate_hand_trace():
    """Sec. 7.6: the removable time counts each record once.
      0 H2D  h->0 [0, 2]    content x; overwritten by record 2 before the kernel: unused (2 ns)
      1 D2H  0->h [10, 15]  content x back: a round-trip return leg (5 ns)
      2 H2D  h->0 [20, 25]  content x again: a duplicate and a return leg (5 ns, once)
      3 KERNEL 0  [26, 30]
      4 ALLOC  0  [30, 33]  touched by the kernel's end: used, and the first of its key
      5 DELETE 0  [34, 38]
      6 H2D  h->0 [40, 46]  content y after the last kernel: unused (6 ns)
      7 ALLOC  0  [50, 51]  same variable again: repeated and unused (1 ns
      8 DELETE 0  [90, 100]   plus its DELETE's 10 ns)
    Span 0..100, removable 2 + 5 + 5 + 6 + 11 = 29, speedup 100 / 71."""
    ev = W.empty_events(9)
    rows = [(W.H2D, -1, 0, 0, 2), (W.D2H, 0, -1, 10, 15), (W.H2D, -1, 0, 20, 25), (W.KERNEL, -1, 0, 26, 30),
            (W.ALLOC, -1, 0, 30, 33), (W.DELETE, -1, 0, 34, 38), (W.H2D, -1, 0, 40, 46),
            (W.ALLOC, -1, 0, 50, 51), (W.DELETE, -1, 0, 90, 100)]
    for i, (op, s, d, t0, t1) in enumerate(rows):
        ev["op"][i], ev["src_dev"][i], ev["dst_dev"][i], ev["t_start"][i], ev["t_end"][i] = op, s, d, t0, t1
    ev["digest"][:3] = 0x77
    ev["digest"][6] = 0x78
    ev["src_addr"][[0, 2]] = W.HOST_BASE
    ev["src_addr"][6] = W.HOST_BASE + 64
    ev["src_addr"][[4, 5, 7, 8]] = W.HOST_BASE + 128
    ev["dst_addr"][[4, 5, 7, 8]] = W.DEV_BASE + 128
    ev["bytes"] = 8
    flags, rep = oracle.analyze(ev)
    want = [oracle.F_UT | oracle.F_RT_TX, oracle.F_RT_TX | oracle.F_RT_RX, oracle.F_DD | oracle.F_RT_RX, 0,
            oracle.F_PAIRED, oracle.F_PAIRED, oracle.F_UT, oracle.F_PAIRED | oracle.F_RA | oracle.F_UA,
            oracle.F_PAIRED]
    assert flags.tolist() == want
    assert rep["elim_ns"] == 29 and rep["span_ns"] == 100
    assert rep["predicted_speedup"] == 100 / 71


def test_savings_estimate_degenerate_spans():
    ev = W.empty_events(1)
    ev["op"], ev["dst_dev"], ev["src_dev"] = W.H2D, 0, -1
    flags, rep = oracle.analyze(ev)  # one zero-length unused copy
    assert rep["span_ns"] == 0 and rep["predicted_speedup"] == 1.0 and flags[0] & oracle.F_UT
    ev["t_end"] = 5
    flags, rep = oracle.analyze(ev)  # everything is removable
    assert rep["elim_ns"] == 5 and rep["predicted_speedup"] == float("inf")
    flags, rep = oracle.analyze(W.empty_events(0))
    assert rep["span_ns"] == 0 and rep["elim_ns"] == 0 and rep["predicted_speedup"] == 1.0


def test_plain_small_planted_subset_of_flags():
    ps = W.PlainSmall(seed=1)
    dg = [oracle.d64(s) for s in ps.snapshots]
    ev = ps.events.copy()
    for i in range(len(ev)):
        if ps.snapshot_of[i] >= 0:
            ev["digest"][i] = dg[ps.snapshot_of[i]]
    flags, rep = oracle.analyze(ev)
    assert rep["status"] == 0
    assert all(flags[i] & oracle.F_DD for i in ps.planted_dd)
    assert all(flags[i] & oracle.F_RT_RX for i in ps.planted_rt_rx)
    assert all(flags[i] & oracle.F_RT_TX for i in ps.planted_rt_tx)
    # byte-level brute force agrees on the whole 1,000-record log
    bflags, bc = brute(ps.events, lambda i: ps.snapshots[ps.snapshot_of[i]].tobytes())
    assert flags.tolist() == bflags


def test_large_arrays_planted_duplicates_exact():
    la = W.LargeArrays(seed=2, n_arrays=4, n_elem=1 << 12, resends=3, device="cpu")
    ev = la.events.copy()
    ev["digest"] = [oracle.d64(s.numpy().view(np.uint8)) for s in la.snapshots]
    flags, rep = oracle.analyze(ev)
    assert rep["dd_events"] == la.planted_dd
    assert [bool(f & oracle.F_DD) for f in flags] == la.identical
