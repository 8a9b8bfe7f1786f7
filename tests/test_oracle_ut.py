"""Pins of the oracle's unused-transfer rule (Def. 4, transfer half; Alg. 5).

Three independent routes: traces worked by hand from the definition, an
O(n^2) brute force that decides "overwritten before any kernel can read it" by
scanning every later transfer, and the paper's Algorithm 5 taken step by step
(pointer and candidate map), which must agree with the rule wherever kernels
on a device do not overlap.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from paper_2601_12713_amd import workloads as W

from brute import _valid, H2D, D2D, KERNEL


def brute_ut(ev):
    n = len(ev)
    valid = [_valid(ev, i) for i in range(n)]
    op = [int(ev[i]["op"]) for i in range(n)]
    dst = [int(ev[i]["dst_dev"]) for i in range(n)]
    src = [int(ev[i]["src_dev"]) for i in range(n)]
    saddr = [int(ev[i]["src_addr"]) for i in range(n)]
    ts = [int(ev[i]["t_start"]) for i in range(n)]
    te = [int(ev[i]["t_end"]) for i in range(n)]
    kernels = {}
    for i in range(n):
        if valid[i] and op[i] == KERNEL:
            kernels.setdefault(dst[i], []).append(i)
    into = [i for i in range(n) if valid[i] and op[i] in (H2D, D2D) and dst[i] >= 0]

    def passed(i):  # kernels on the transfer's device that ended before it started
        return sum(1 for k in kernels.get(dst[i], []) if te[k] < ts[i])

    def in_gap(i, e):
        K = kernels.get(dst[i], [])
        return e < len(K) and ts[K[e]] > ts[i]

    ut = [0] * n
    for i in into:
        e = passed(i)
        if e == len(kernels.get(dst[i], [])):
            ut[i] = 1
        elif in_gap(i, e):
            for j in into:
                if (j > i and dst[j] == dst[i] and src[j] == src[i] and saddr[j] == saddr[i]
                        and passed(j) == e and in_gap(j, e)):
                    ut[i] = 1
                    break
    return ut


def trace(rows):
    """rows: (op, src_dev, dst_dev, src_addr, t_start, t_end)."""
    ev = W.empty_events(len(rows))
    for i, (op, s, d, a, t0, t1) in enumerate(rows):
        ev["op"][i], ev["src_dev"][i], ev["dst_dev"][i] = op, s, d
        ev["src_addr"][i], ev["dst_addr"][i] = a, W.DEV_BASE + a
        ev["t_start"][i], ev["t_end"][i] = t0, t1
        ev["bytes"][i] = 64
    return ev


A, B = W.HOST_BASE, W.HOST_BASE + 4096


def test_overwritten_before_the_kernel():
    # Two copies of host A to device 0, then a kernel: the first copy is
    # overwritten before the kernel could read it.
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.H2D, -1, 0, A, 10, 15), (W.KERNEL, -1, 0, 0, 20, 30)])
    assert oracle.unused_transfers(ev).tolist() == [1, 0, 0]


def test_kernel_between_copies_may_have_read_the_first():
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.H2D, -1, 0, A, 30, 35),
                (W.KERNEL, -1, 0, 0, 40, 50)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0]


def test_copy_after_the_last_kernel_is_unused():
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.H2D, -1, 0, B, 30, 35)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 1]


def test_device_without_kernels():
    # Nothing ever runs on device 1: every copy to it is unused; the copy to
    # device 0 is read by device 0's kernel.
    ev = trace([(W.H2D, -1, 1, A, 0, 5), (W.H2D, -1, 0, A, 6, 8), (W.KERNEL, -1, 0, 0, 10, 20)])
    assert oracle.unused_transfers(ev).tolist() == [1, 0, 0]


def test_copies_back_to_the_host_are_never_unused():
    # A D2H after the last kernel is the usual copy of results (reading: the
    # rule covers data mapped to a device only).
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.D2H, 0, -1, W.DEV_BASE, 30, 35),
                (W.D2H, 0, -1, W.DEV_BASE, 40, 45)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0]


def test_copy_overlapping_a_kernel_clears_the_candidates():
    # The second copy overlaps the running kernel (it may be read by it), so it
    # is no candidate; the first copy was in the gap before that kernel and is
    # the last of its address there.
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 40), (W.H2D, -1, 0, A, 20, 25),
                (W.KERNEL, -1, 0, 0, 50, 60)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0]


def test_different_addresses_and_devices_do_not_overwrite():
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.H2D, -1, 0, B, 6, 8), (W.H2D, -1, 1, A, 9, 10),
                (W.KERNEL, -1, 0, 0, 20, 30), (W.KERNEL, -1, 1, 0, 20, 30)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0, 0]


def test_device_to_device_copies_key_on_their_source_device():
    # Device 1 address A and host address A are different memory: no overwrite.
    # Two copies from device 1 address A into device 0: the first is unused.
    ev = trace([(W.D2D, 1, 0, A, 0, 5), (W.H2D, -1, 0, A, 6, 8), (W.D2D, 1, 0, A, 9, 10),
                (W.KERNEL, -1, 0, 0, 20, 30)])
    assert oracle.unused_transfers(ev).tolist() == [1, 0, 0, 0]


def test_repeated_copies_closed_form():
    # m copies of one address in the gap before a kernel: m - 1 unused.
    for m in range(1, 9):
        rows = [(W.H2D, -1, 0, A, 10 * i, 10 * i + 5) for i in range(m)] + [(W.KERNEL, -1, 0, 0, 1000, 1010)]
        u = oracle.unused_transfers(trace(rows))
        assert int(u.sum()) == m - 1 and u[m - 1] == 0


def test_empty_log():
    assert oracle.unused_transfers(W.empty_events(0)).tolist() == []


@settings(max_examples=200, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n_dev=st.integers(1, 3), n=st.integers(1, 60))
def test_rule_matches_brute_force(seed, n_dev, n):
    ev, _, _ = W.tiny_trace(seed, n_events=n, n_devices=n_dev, n_vars=3)
    assert oracle.unused_transfers(ev).tolist() == brute_ut(ev)


@settings(max_examples=150, deadline=None)
@given(seed=st.integers(0, 2**32 - 1))
def test_rule_matches_brute_force_invalid_and_overlapping(seed):
    ev, _, _ = W.tiny_trace(seed, n_events=50, n_devices=2, n_vars=3, invalid_rate=0.15)
    assert oracle.unused_transfers(ev).tolist() == brute_ut(ev)
    ev, _, _ = W.tiny_trace(seed, n_events=50, n_devices=2, n_vars=3, overlap_kernels=True)
    assert oracle.unused_transfers(ev).tolist() == brute_ut(ev)


def _kernels_overlap(ev, K):
    by_dev = {}
    for k in K:
        by_dev.setdefault(int(ev["dst_dev"][k]), []).append(k)
    for ks in by_dev.values():
        for a, b in zip(ks, ks[1:]):
            if int(ev["t_start"][b]) <= int(ev["t_end"][a]):
                return True
    return False


@settings(max_examples=200, deadline=None)
@given(seed=st.integers(0, 2**32 - 1), n_dev=st.integers(1, 3))
def test_algorithm5_matches_rule_without_overlapping_kernels(seed, n_dev):
    ev, _, _ = W.tiny_trace(seed, n_events=60, n_devices=n_dev, n_vars=3)
    valid = [_valid(ev, i) for i in range(len(ev))]
    K = [i for i in range(len(ev)) if valid[i] and int(ev["op"][i]) == KERNEL]
    if _kernels_overlap(ev, K):
        return
    T = [i for i in range(len(ev)) if valid[i] and int(ev["op"][i]) in (H2D, D2D) and int(ev["dst_dev"][i]) >= 0]
    rule = oracle.unused_transfers(ev)
    alg = oracle.alg5(ev, np.array(K, dtype=np.uint64), np.array(T, dtype=np.uint64))
    assert alg.tolist() == [int(rule[i]) for i in T]


def test_algorithm5_and_rule_on_planted_trace():
    # The hand trace of the first case, through the step-by-step algorithm.
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.H2D, -1, 0, A, 10, 15), (W.KERNEL, -1, 0, 0, 20, 30),
                (W.H2D, -1, 0, A, 40, 45)])
    alg = oracle.alg5(ev, np.array([2], dtype=np.uint64), np.array([0, 1, 3], dtype=np.uint64))
    assert alg.tolist() == [1, 0, 1]
    assert oracle.unused_transfers(ev).tolist() == [1, 0, 0, 1]
