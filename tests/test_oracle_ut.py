"""Pins of the oracle's unused-transfer rule (Def. 4, transfer half; Alg. 5).

Two independent routes: traces worked by hand from the definition (each case
of the paper's description of Alg. 5: a copy overwritten in the gap before a
kernel, a kernel in between, a copy after the last kernel, a device without
kernels, a copy overlapping a running kernel), and the brute force of
tests/brute.py, which decides "read by some kernel before a later copy to the
same place begins" by quantifying over every kernel and every later copy.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from paper_2601_12713_amd import workloads as W

from brute import brute, F_UT


def brute_ut(ev):
    flags, _ = brute(ev, lambda i: b"")
    return [1 if f & F_UT else 0 for f in flags]


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


def test_overlapping_kernels():
    # Two kernels on device 0 overlap: [10, 100] and [20, 30]. A copy at 40
    # is read by the long kernel still running (it meets [40, 50]); the copy
    # at 50 is overwritten at 60 with no kernel starting in between, but the
    # long kernel runs across both, so it may read either: used.
    ev = trace([(W.KERNEL, -1, 0, 0, 10, 100), (W.KERNEL, -1, 0, 0, 20, 30), (W.H2D, -1, 0, A, 40, 45),
                (W.H2D, -1, 0, A, 50, 55), (W.H2D, -1, 0, A, 60, 65), (W.H2D, -1, 0, B, 110, 115)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0, 0, 1]


def test_touching_ends_count_as_use():
    # A kernel ending exactly when the copy starts, or starting exactly when
    # the overwrite starts, may read the copy (closed intervals).
    ev = trace([(W.KERNEL, -1, 0, 0, 0, 10), (W.H2D, -1, 0, A, 10, 12), (W.H2D, -1, 0, A, 14, 16),
                (W.KERNEL, -1, 0, 0, 14, 20)])
    assert oracle.unused_transfers(ev).tolist() == [0, 0, 0, 0]
    ev = trace([(W.KERNEL, -1, 0, 0, 0, 9), (W.H2D, -1, 0, A, 10, 12), (W.H2D, -1, 0, A, 14, 16),
                (W.KERNEL, -1, 0, 0, 15, 20)])
    assert oracle.unused_transfers(ev).tolist() == [0, 1, 0, 0]


def test_report_counts_and_sums_of_unused_transfers():
    ev = trace([(W.H2D, -1, 0, A, 0, 5), (W.H2D, -1, 0, A, 10, 17), (W.KERNEL, -1, 0, 0, 20, 30),
                (W.H2D, -1, 0, B, 40, 49)])
    ev["bytes"] = [100, 200, 0, 300]
    flags, rep = oracle.analyze(ev)
    assert rep["ut_events"] == 2 and rep["ut_bytes"] == 400 and rep["ut_time_ns"] == 5 + 9
