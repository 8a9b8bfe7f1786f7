"""Oracle parity at each configuration's full shape, the sizes bench.py times,
through the C ABI. The plain-small log and the 10^7-record trace are checked
whole in test_gpu_analyze.py; here:
  large arrays  all 64 digests of the 16 x 256 MiB fp64 transfers, both forms
  batch         all 100,000 digests of the 48e9-byte batch, from the
                graph-replayed batched launch under the saved tuning
  serving       a 200k requests/s schedule of 4 KiB-64 MiB payloads over a
                16 GiB arena: served digests, final flags and report against
                the oracle on the arrival-ordered log, sampled requests alone
                against the mix; and a burst of 64 MiB payloads at t = 0 whose
                admission waits on the byte budget.
The oracle runs on the host's cores, one buffer per task."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

from gpu_helpers import compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WORKERS = min(16, os.cpu_count() or 1)


def oracle_many(host_views):
    """D64 of each host byte array, computed in parallel (the oracle call releases the GIL)."""
    with ThreadPoolExecutor(WORKERS) as ex:
        return np.array(list(ex.map(oracle.d64, host_views)), dtype=np.uint64)


def test_large_arrays_all_digests(odp):
    la = W.LargeArrays(seed=2, device="cuda")
    la.materialize()
    plain = odp.digest_tensors(la.snapshots, plain=True)
    batched = odp.digest_tensors(la.snapshots)
    want = np.zeros(len(la.snapshots), dtype=np.uint64)
    for g in range(0, len(la.snapshots), 16):  # 4 GiB of host copies at a time
        host = [s.cpu().numpy().view(np.uint8) for s in la.snapshots[g:g + 16]]
        want[g:g + 16] = oracle_many(host)
        del host
    assert (plain == want).all(), np.nonzero(plain != want)[0][:8]
    assert (batched == want).all(), np.nonzero(batched != want)[0][:8]
    ev = la.events.copy()
    ev["digest"] = want
    fo, ro = oracle.analyze(ev)
    assert ro["dd_events"] == la.planted_dd
    del la
    torch.cuda.empty_cache()


def test_batch_all_digests(odp):
    bb = W.BatchBuffers(seed=3, device="cuda")
    n = bb.sizes.size
    dptr = torch.tensor(bb.pointers().view(np.int64), device="cuda")
    dsz = torch.tensor(bb.sizes.view(np.int64), device="cuda")
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    assert odp.get_tuning()["use_graph"] == 1
    odp.reserve(max_buffers=n, max_total_bytes=int(bb.total_bytes))
    for _ in range(2):  # capture, then a replay
        out.fill_(-1)
        odp.digest_buffers(dptr, dsz, out)
        torch.cuda.synchronize()
    assert odp.device_status() == odp.ODP_OK
    got = out.cpu().numpy().view(np.uint64)
    want = np.zeros(n, dtype=np.uint64)
    # stream the arena through one pinned host block, ~1 GiB of whole buffers at a time
    block = torch.empty((1 << 30) + (64 << 20), dtype=torch.uint8, pin_memory=True)
    hb = block.numpy()
    i = 0
    while i < n:
        o0 = int(bb.offsets[i])
        j = i
        while j < n and int(bb.offsets[j]) + int(bb.sizes[j]) - o0 <= block.numel():
            j += 1
        assert j > i
        o1 = int(bb.offsets[j - 1]) + int(bb.sizes[j - 1])
        block[:o1 - o0].copy_(bb.arena[o0:o1])
        views = [hb[int(bb.offsets[k]) - o0:int(bb.offsets[k]) - o0 + int(bb.sizes[k])] for k in range(i, j)]
        want[i:j] = oracle_many(views)
        i = j
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%d of %d digests differ, first %s" % (bad.size, n, bad[:8].tolist())
    cp = bb.copy_of >= 0
    assert (want[cp] == want[bb.copy_of[cp]]).all()
    del bb, block
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def arena16(odp):
    gib = 1 << 30
    a = torch.empty(16 * gib, dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for off in range(0, a.numel(), gib):
        a[off:off + gib].copy_(torch.randint(0, 256, (gib,), dtype=torch.uint8, device="cuda", generator=gen))
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


def oracle_payload_digests(sched, arena):
    ev = sched.events.copy()
    keys = sorted({(int(o), int(b)) for o, b in zip(sched.payload_off, sched.payload_bytes) if o >= 0})

    def one(key):
        o, b = key
        return oracle.d64(arena[o:o + b].cpu().numpy())

    with ThreadPoolExecutor(WORKERS) as ex:
        dg = dict(zip(keys, ex.map(one, keys)))
    for i in np.nonzero(sched.payload_off >= 0)[0]:
        ev["digest"][i] = dg[(int(sched.payload_off[i]), int(sched.payload_bytes[i]))]
    return ev


def serve_and_check(odp, sched, arena, budget, sample=40):
    srv = odp.Server(max_events=len(sched.events), budget_bytes=budget)
    done, stats = srv.run(sched.events, sched.payload_ptrs(), sched.payload_bytes, sched.arrival_ns)
    log = srv.log().view(W.EVENT_DTYPE)
    imm, fl, rep = srv.drain()
    srv.close()
    ev_o = oracle_payload_digests(sched, arena)
    tx = sched.payload_off >= 0
    assert (log["digest"][tx] == ev_o["digest"][tx]).all(), "served digests differ from the oracle"
    fo, ro = oracle.analyze(ev_o)
    compare(fl, rep, fo, ro)
    rng = np.random.default_rng(9)
    for i in rng.choice(np.nonzero(tx)[0], size=min(sample, int(tx.sum())), replace=False):
        o, b = int(sched.payload_off[i]), int(sched.payload_bytes[i])
        assert odp.digest_tensors([arena[o:o + b]])[0] == log["digest"][i], i
    return stats, ro


def test_serving_200k_per_s_full_payloads(odp, arena16):
    sched = W.ServingSchedule(seed=6, n=2000, rate=200_000.0, lo=4096, hi=64 << 20, arena=arena16)
    stats, ro = serve_and_check(odp, sched, arena16, budget=16 << 30)
    assert stats["bytes"] == int(sched.payload_bytes.sum()) and stats["max_tick"] > 1
    assert ro["dd_events"] > 100 and ro["rt_rx_events"] > 0 and ro["n_alloc_pairs"] > 0


def test_serving_burst_of_64MiB_payloads(odp, arena16):
    sched = W.ServingSchedule(seed=7, n=150, rate=1e9, lo=64 << 20, hi=64 << 20, arena=arena16)
    sched.arrival_ns[:] = 0
    stats, ro = serve_and_check(odp, sched, arena16, budget=1 << 30, sample=10)
    # a tick holds at most 16 payloads of 64 MiB (plus records that carry none)
    payloads = int((sched.payload_bytes > 0).sum())
    assert stats["budget_waits"] > 0 and stats["ticks"] >= payloads // 16
