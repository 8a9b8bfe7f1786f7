"""Pins of the oracle's detection rules against things other than itself:
brute force over the paper's definitions with byte equality (tests/brute.py),
the worked examples of the paper's Listings 1 and 2 (tests/golden/), closed
forms, and the paper's Algorithms 1-4 taken step by step.
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
        assert rep[k] == v, k
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


@settings(max_examples=200, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n_dev=st.integers(1, 3))
def test_algorithm1_groups_match_duplicate_rule(seed, n_dev):
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=60, n_devices=n_dev)
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    T = _valid_transfers(evd, flags)
    ng, group_of = oracle.alg1(evd, T)
    assert ng == rep["dd_groups"]
    assert int((group_of >= 0).sum()) == rep["dd_members"]
    seen = set()
    for k, i in enumerate(T):
        g = int(group_of[k])
        is_dup = g >= 0 and g in seen
        seen.add(g)
        assert bool(flags[i] & oracle.F_DD) == is_dup


@settings(max_examples=300, deadline=None)
@given(seed=st.integers(0, 2**32 - 1))
def test_algorithm2_matches_round_trip_rule_on_two_endpoints(seed):
    """With two endpoints per content, Algorithm 2's recorded <tx, rx> pairs are
    exactly the RT_TX records, each paired with the first later reversed record,
    and the rx records are exactly the RT_RX records."""
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=60, n_devices=1, n_payloads=4)
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    T = [i for i in _valid_transfers(evd, flags) if evd["src_dev"][i] != evd["dst_dev"][i]]
    pairs = oracle.alg2(evd, np.array(T, dtype=np.uint64))
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
    pairs = oracle.alg2(ev, np.array([0, 1], dtype=np.uint64))
    assert pairs == [(1, 0)]


def _pairs(evd, flags):
    AD = [i for i in range(len(evd)) if evd["op"][i] in (W.ALLOC, W.DELETE) and flags[i] & oracle.F_PAIRED]
    allocs = [i for i in AD if evd["op"][i] == W.ALLOC]
    dels = []
    for a in allocs:
        nxt = [j for j in AD if j > a and evd["dst_dev"][j] == evd["dst_dev"][a] and evd["dst_addr"][j] == evd["dst_addr"][a]]
        dels.append(nxt[0])
    return np.array(allocs, dtype=np.uint64), np.array(dels, dtype=np.uint64)


@settings(max_examples=200, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n_dev=st.integers(1, 3))
def test_algorithm3_and_4_match_allocation_rules(seed, n_dev):
    ev, payloads, payload_of = W.tiny_trace(seed, n_events=60, n_devices=n_dev, n_vars=3)
    evd = with_digests(ev, payloads, payload_of)
    flags, rep = oracle.analyze(evd)
    ai, di = _pairs(evd, flags)
    ng, rank = oracle.alg3(evd, ai, di)
    assert ng == rep["ra_groups"]
    assert [bool(flags[a] & oracle.F_RA) for a in ai] == [r >= 1 for r in rank]
    K = np.array([i for i in range(len(evd)) if evd["op"][i] == W.KERNEL and not flags[i] & oracle.F_INVALID], dtype=np.uint64)
    unused = oracle.alg4(evd, K, ai, di)
    assert [bool(flags[a] & oracle.F_UA) for a in ai] == [bool(u) for u in unused]


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
        assert rep[k] == v, k
    assert rep["status"] == 0


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
