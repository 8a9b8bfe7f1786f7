"""GPU parity of the literal Algorithm 2 comparison mode (Sec. 5, Alg. 2) with
the oracle's restatement of the algorithm: the same <tx, rx> pairs on logs
with two and more endpoints, and the same flags and report as the analysis."""
import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

from gpu_helpers import compare
from test_gpu_analyze import with_digests

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NONE = 0xFFFFFFFF


def alg2_gpu(odp, ev):
    n = len(ev)
    raw = np.ascontiguousarray(ev).view(np.uint8).reshape(-1)
    d_ev = torch.from_numpy(raw.copy()).to("cuda") if n else torch.zeros(64, dtype=torch.uint8, device="cuda")
    d_flags = torch.full((max(n, 1),), 0xAA, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    d_rx = torch.full((max(n, 1),), 7, dtype=torch.int32, device="cuda")
    d_np = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
    odp.analyze_trace_alg2(d_ev, d_flags, d_rep, d_rx, d_np, n=n)
    torch.cuda.synchronize()
    rx = d_rx[:n].cpu().numpy().view(np.uint32)
    return d_flags[:n].cpu().numpy(), odp.report_to_dict(d_rep.cpu().numpy()), rx, int(d_np.item())


def valid_transfers(ev, flags):
    return np.nonzero(((ev["op"] == W.H2D) | (ev["op"] == W.D2H) | (ev["op"] == W.D2D)) &
                      ((flags & oracle.F_INVALID) == 0))[0]


def expected_rx(ev, T):
    rx = np.full(len(ev), NONE, dtype=np.uint32)
    pairs = oracle.alg2_pairs(ev, T.astype(np.uint64))
    for t, r in pairs:
        rx[T[t]] = T[r]
    return rx, len(pairs)


def check(odp, ev, transfers=None):
    """transfers: the valid transfers when the log is valid by construction
    (the oracle's analysis is then skipped), else None."""
    fg, rg, rx, npairs = alg2_gpu(odp, ev)
    if transfers is None:
        fr, rr = oracle.analyze(ev)
        compare(fg, rg, fr, rr)
        transfers = valid_transfers(ev, fr)
    want, nwant = expected_rx(ev, transfers)
    bad = np.nonzero(rx != want)[0]
    assert bad.size == 0, "rx differs at %s: gpu %s oracle %s" % (bad[:8].tolist(), rx[bad[:8]].tolist(),
                                                                    want[bad[:8]].tolist())
    assert npairs == nwant
    return rx, npairs, rg


def test_return_leg_from_a_third_endpoint(odp):
    """dev1 -> host, then host -> dev0, one content: Algorithm 2 records the
    second with the first as its rx (the rule sees no round trip)."""
    ev = W.empty_events(2)
    ev["op"] = [W.D2H, W.H2D]
    ev["src_dev"], ev["dst_dev"] = [1, -1], [-1, 0]
    ev["t_start"], ev["t_end"] = [0, 10], [5, 15]
    ev["digest"] = 77
    rx, npairs, rep = check(odp, ev)
    assert rx.tolist() == [NONE, 0] and npairs == 1 and rep["rt_pairs"] == 0


def test_empty_and_one_record(odp):
    rx, npairs, _ = check(odp, W.empty_events(0))
    assert npairs == 0
    ev = W.empty_events(1)
    ev["op"] = W.H2D
    ev["src_dev"], ev["dst_dev"] = 0, 0     # a self-transfer is its own rx
    ev["digest"] = 5
    rx, npairs, _ = check(odp, ev)
    assert rx.tolist() == [0] and npairs == 1


@pytest.mark.parametrize("n_devices", [1, 3, 10])
def test_random_small_traces(odp, n_devices):
    """Random logs over host + 1, 3 and 10 devices (rejected records, ties,
    repeated and one-bit-apart contents), lengths across the one-workgroup
    thresholds of the analysis."""
    for seed in range(12):
        n = [40, 300, 700, 2500][seed % 4]
        ev, payloads, payload_of = W.tiny_trace(900 + 31 * seed + n_devices, n_events=n, n_devices=n_devices,
                                                n_payloads=5, invalid_rate=0.02 if seed % 3 == 0 else 0.0)
        check(odp, with_digests(ev, payloads, payload_of))


def test_two_endpoints_give_the_round_trips(odp):
    """On one device and the host, the recorded pairs are the round trips:
    their number is rt_pairs and their tx records are the RT_TX ones."""
    ev, payloads, payload_of = W.tiny_trace(77, n_events=2000, n_devices=1, n_payloads=6)
    ev = with_digests(ev, payloads, payload_of)
    T = set(valid_transfers(ev, oracle.analyze(ev)[0]).tolist())
    ev = ev[[i for i in range(len(ev)) if not (i in T and ev["src_dev"][i] == ev["dst_dev"][i])]]
    rx, npairs, rep = check(odp, ev)
    fr, _ = oracle.analyze(ev)
    assert npairs == rep["rt_pairs"]
    assert sorted(np.nonzero(rx != NONE)[0].tolist()) == sorted(np.nonzero(fr & oracle.F_RT_TX)[0].tolist())


def test_many_tiles_many_endpoints(odp):
    """60,000 records over host + 10 devices: groups of one record (some
    self-transfers), groups of hundreds that span many wavefronts' positions,
    the all-ones digest shared with non-transfers, rejected records."""
    rng = np.random.default_rng(5)
    m = 60_000
    ev = W.empty_events(m)
    op = rng.choice([W.H2D, W.D2H, W.D2D, W.ALLOC, W.KERNEL, W.DELETE], size=m, p=[0.3, 0.25, 0.25, 0.08, 0.07, 0.05])
    ev["op"] = op
    src = rng.integers(-1, 10, size=m)
    dst = rng.integers(-1, 10, size=m)
    dst = np.where(op == W.H2D, np.maximum(dst, 0), dst)
    src = np.where(op == W.H2D, -1, src)
    dst = np.where(op == W.D2H, -1, dst)
    src = np.where(op == W.D2H, np.maximum(src, 0), src)
    ev["src_dev"], ev["dst_dev"] = src, dst
    ev["t_start"] = np.arange(m, dtype=np.uint64) * 2
    ev["t_end"] = ev["t_start"] + 1
    hot = rng.integers(0, 2**63, size=40, dtype=np.uint64)
    dig = np.where(rng.random(m) < 0.6, rng.choice(hot, size=m), rng.integers(0, 2**63, size=m, dtype=np.uint64))
    dig = np.where(rng.random(m) < 0.01, np.uint64(0xFFFFFFFFFFFFFFFF), dig)
    ev["digest"] = dig
    bad = rng.random(m) < 0.002
    ev["t_end"] = np.where(bad, ev["t_start"] - np.uint64(1), ev["t_end"])
    rx, npairs, _ = check(odp, ev)
    assert npairs > 10_000


def test_log_above_packed_index_limit(odp):
    """2^24 + 5,000 records (record indices no longer fit beside the endpoint
    codes in the sort's values): a few thousand transfers among allocations."""
    rng = np.random.default_rng(8)
    m = (1 << 24) + 5000
    ev = W.empty_events(m)
    ev["op"] = W.ALLOC
    ev["dst_dev"] = 0
    ev["bytes"] = 64
    ev["dst_addr"] = np.uint64(W.DEV_BASE) + (np.arange(m, dtype=np.uint64) << np.uint64(6))
    ev["t_start"] = np.arange(m, dtype=np.uint64)
    ev["t_end"] = ev["t_start"]
    tx = np.sort(rng.choice(m, size=6000, replace=False))
    ev["op"][tx] = rng.choice([W.H2D, W.D2H, W.D2D], size=tx.size)
    ev["src_dev"][tx] = rng.integers(0, 3, size=tx.size)
    ev["dst_dev"][tx] = rng.integers(0, 3, size=tx.size)
    h2d, d2h = ev["op"][tx] == W.H2D, ev["op"][tx] == W.D2H
    ev["src_dev"][tx[h2d]] = -1
    ev["dst_dev"][tx[d2h]] = -1
    ev["digest"][tx] = rng.integers(0, 50, size=tx.size).astype(np.uint64)
    rx, npairs, rep = check(odp, ev, transfers=tx)
    assert rep["n_transfers"] == tx.size and npairs > 1000
