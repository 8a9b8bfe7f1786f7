"""GPU parity of the unused-transfer rule (Def. 4, transfer half; Alg. 5) and
of the optimization-potential estimate (Sec. 7.6) against the CPU oracle,
through the C ABI: the hand traces that pin the oracle, run through each of
the analysis's three code paths (one workgroup up to 512 records, one-workgroup
sorts up to 2,048, multi-launch passes above), and random logs that spread
copies of few source addresses over many tiles."""
import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

from gpu_helpers import analyze_gpu, compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

A, B = W.HOST_BASE, W.HOST_BASE + 4096

# (op, src_dev, dst_dev, src_addr, t_start, t_end): each case of the rule
HAND_TRACES = {
    "overwritten_before_kernel": [(W.H2D, -1, 0, A, 0, 5), (W.H2D, -1, 0, A, 10, 15), (W.KERNEL, -1, 0, 0, 20, 30)],
    "kernel_between": [(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.H2D, -1, 0, A, 30, 35),
                       (W.KERNEL, -1, 0, 0, 40, 50)],
    "after_last_kernel": [(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.H2D, -1, 0, B, 30, 35)],
    "device_without_kernels": [(W.H2D, -1, 1, A, 0, 5), (W.H2D, -1, 0, A, 6, 8), (W.KERNEL, -1, 0, 0, 10, 20)],
    "d2h_never_unused": [(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 20), (W.D2H, 0, -1, W.DEV_BASE, 30, 35),
                         (W.D2H, 0, -1, W.DEV_BASE, 40, 45)],
    "overlapping_running_kernel": [(W.H2D, -1, 0, A, 0, 5), (W.KERNEL, -1, 0, 0, 10, 40), (W.H2D, -1, 0, A, 20, 25),
                                   (W.KERNEL, -1, 0, 0, 50, 60)],
    "d2d_keys_on_source_device": [(W.D2D, 1, 0, A, 0, 5), (W.H2D, -1, 0, A, 6, 8), (W.D2D, 1, 0, A, 9, 10),
                                  (W.KERNEL, -1, 0, 0, 20, 30)],
    "overlapping_kernels": [(W.KERNEL, -1, 0, 0, 10, 100), (W.KERNEL, -1, 0, 0, 20, 30), (W.H2D, -1, 0, A, 40, 45),
                            (W.H2D, -1, 0, A, 50, 55), (W.H2D, -1, 0, A, 60, 65), (W.H2D, -1, 0, B, 110, 115)],
    "touching_ends_used": [(W.KERNEL, -1, 0, 0, 0, 10), (W.H2D, -1, 0, A, 10, 12), (W.H2D, -1, 0, A, 14, 16),
                           (W.KERNEL, -1, 0, 0, 14, 20)],
    "touching_ends_gap": [(W.KERNEL, -1, 0, 0, 0, 9), (W.H2D, -1, 0, A, 10, 12), (W.H2D, -1, 0, A, 14, 16),
                          (W.KERNEL, -1, 0, 0, 15, 20)],
}
# the oracle's hand-worked answers (tests/test_oracle_ut.py)
EXPECT_UT = {
    "overwritten_before_kernel": [1, 0, 0], "kernel_between": [0, 0, 0, 0], "after_last_kernel": [0, 0, 1],
    "device_without_kernels": [1, 0, 0], "d2h_never_unused": [0, 0, 0, 0], "overlapping_running_kernel": [0, 0, 0, 0],
    "d2d_keys_on_source_device": [1, 0, 0, 0], "overlapping_kernels": [0, 0, 0, 0, 0, 1],
    "touching_ends_used": [0, 0, 0, 0], "touching_ends_gap": [0, 1, 0, 0],
}


def trace(rows):
    ev = W.empty_events(len(rows))
    for i, (op, s, d, a, t0, t1) in enumerate(rows):
        ev["op"][i], ev["src_dev"][i], ev["dst_dev"][i] = op, s, d
        ev["src_addr"][i], ev["dst_addr"][i] = a, W.DEV_BASE + a
        ev["t_start"][i], ev["t_end"][i] = t0, t1
        ev["bytes"][i] = 64 + 8 * i
    return ev


def padded(ev, total):
    """The log followed by KERNEL records on device 9 (which no case uses), so
    that it takes the code path of a `total`-record log with the same
    answers for the original records."""
    if total <= len(ev):
        return ev
    pad = W.empty_events(total - len(ev))
    t0 = int(ev["t_start"].max()) if len(ev) else 0
    pad["op"], pad["dst_dev"], pad["src_dev"] = W.KERNEL, 9, -1
    pad["t_start"] = t0 + np.arange(pad.size, dtype=np.uint64)
    pad["t_end"] = pad["t_start"]
    return np.concatenate([ev, pad])


def check(odp, ev):
    fr, rr = oracle.analyze(ev)
    fg, rg = analyze_gpu(odp, ev)
    compare(fg, rg, fr, rr)
    return fg, rg


@pytest.mark.parametrize("total", [0, 600, 3000])
@pytest.mark.parametrize("name", sorted(HAND_TRACES))
def test_hand_traces_every_path(odp, name, total):
    ev = padded(trace(HAND_TRACES[name]), total)
    fg, rg = check(odp, ev)
    m = len(HAND_TRACES[name])
    assert [1 if f & odp.F_UT else 0 for f in fg[:m]] == EXPECT_UT[name]


def savings_trace():
    """The hand trace of the savings estimate: span 100 ns, 29 ns removable."""
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
    return ev


def test_savings_estimate_hand_trace(odp):
    fg, rg = check(odp, savings_trace())
    assert rg["elim_ns"] == 29 and rg["span_ns"] == 100 and rg["predicted_speedup"] == 100 / 71


@pytest.mark.parametrize("total", [600, 3000])
def test_savings_estimate_long_paths(odp, total):
    """The same trace in longer logs: the padding kernels stretch the span and
    remove nothing."""
    ev = padded(savings_trace(), total)
    fg, rg = check(odp, ev)
    assert rg["elim_ns"] == 29 and rg["span_ns"] == 90 + (total - 9) - 1


@pytest.mark.parametrize("total", [1, 600, 3000])
def test_savings_estimate_degenerate_spans(odp, total):
    """Zero span: speedup 1; everything removable: +infinity."""
    ev = W.empty_events(total)
    ev["op"], ev["dst_dev"], ev["src_dev"] = W.H2D, 0, -1
    ev["src_addr"] = W.HOST_BASE + 64 * np.arange(total, dtype=np.uint64)
    ev["digest"] = np.arange(total, dtype=np.uint64)
    fg, rg = check(odp, ev)
    assert rg["span_ns"] == 0 and rg["predicted_speedup"] == 1.0 and rg["ut_events"] == total
    ev["t_end"] = 5
    fg, rg = check(odp, ev)
    assert rg["elim_ns"] == 5 * total and rg["predicted_speedup"] == float("inf")


@pytest.mark.parametrize("seed,n,n_vars,overlap,inv", [
    (1, 5_000, 3, False, 0.0), (2, 50_000, 7, True, 0.0), (3, 300_000, 40, False, 0.02), (4, 300_000, 2, True, 0.01)])
def test_random_logs_many_tiles(odp, seed, n, n_vars, overlap, inv):
    """Copies of a few source addresses into three devices spread over many
    4,096-record tiles (groups far longer than a tile), with overlapping
    kernels or rejected records."""
    ev, _, _ = W.tiny_trace(7000 + seed, n_events=n, n_devices=3, n_payloads=5, n_vars=n_vars,
                            invalid_rate=inv, overlap_kernels=overlap)
    ev["digest"] = np.random.default_rng(seed).integers(0, 50, size=n).astype(np.uint64)
    fg, rg = check(odp, ev)
    assert rg["ut_events"] > 0


def test_copies_from_every_endpoint(odp):
    """D2D and H2D copies from all eleven endpoints into ten devices, source
    addresses from a small pool, kernels on half the devices."""
    rng = np.random.default_rng(12)
    m = 40_000
    ev = W.empty_events(m)
    ev["op"] = rng.choice([W.H2D, W.D2D, W.D2H, W.KERNEL], size=m, p=[0.4, 0.3, 0.1, 0.2])
    ev["src_dev"] = rng.integers(-1, 10, size=m)
    ev["dst_dev"] = np.where(ev["op"] == W.KERNEL, rng.choice([0, 2, 4, 6, 8], size=m), rng.integers(0, 10, size=m))
    ev["src_addr"] = W.HOST_BASE + 4096 * rng.integers(0, 16, size=m).astype(np.uint64)
    ev["digest"] = rng.integers(0, 1000, size=m).astype(np.uint64)
    ev["t_start"] = np.cumsum(rng.integers(0, 4, size=m)).astype(np.uint64)
    ev["t_end"] = ev["t_start"] + rng.integers(0, 6, size=m).astype(np.uint64)
    ev["bytes"] = 64
    fg, rg = check(odp, ev)
    assert rg["ut_events"] > 1000


@pytest.mark.parametrize("every", [40, 500])
def test_long_kernel_epochs(odp, every):
    """Chronological logs whose kernels are far apart: a copy's next copy is
    searched forward among the copies before the next kernel; past 64 copies
    the sorted path decides (switched on by the device). Ties of a copy's start
    with the next kernel's start occur on purpose."""
    rng = np.random.default_rng(every)
    m = 30_000
    ev = W.empty_events(m)
    is_k = (np.arange(m) % every) == every - 1
    ev["op"] = np.where(is_k, W.KERNEL, rng.choice([W.H2D, W.D2H], size=m, p=[0.8, 0.2]))
    ev["src_dev"] = np.where(ev["op"] == W.D2H, 0, -1)
    ev["dst_dev"] = np.where(ev["op"] == W.D2H, -1, rng.integers(0, 2, size=m))
    ev["src_addr"] = W.HOST_BASE + 4096 * rng.integers(0, 5, size=m).astype(np.uint64)
    ev["digest"] = rng.integers(0, 100, size=m).astype(np.uint64)
    ev["t_start"] = np.cumsum(rng.integers(0, 2, size=m)).astype(np.uint64)
    ev["t_end"] = ev["t_start"] + rng.integers(0, 3, size=m).astype(np.uint64)
    ev["bytes"] = 64
    fg, rg = check(odp, ev)
    assert 0 < rg["ut_events"] < rg["n_transfers"]
