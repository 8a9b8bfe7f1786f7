#!/usr/bin/env python3
"""Benchmark of the content-digest and mapping-trace hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line. A step is one pass of the whole hot path over one batch
of synthetic input: every transfer's buffer is digested, the digests are
written into the event log, and the log is analysed (duplicate, round-trip,
repeated and unused mappings). Inputs are resident in HBM before timing.

Workloads (--workload):
  batch         (default) 100,000 buffers, log-uniform 64 B-16 MiB capped at
                48e9 bytes in total, 25% copies; a step digests them with one
                batched launch sequence (hipGraph replay, saved tuning), writes
                the digests into the batch's 101,562-record transfer log and
                analyses it. The per-buffer-launch form of the same buffers,
                the large-arrays workload, the trace analysis and a short
                serving run (50k and 200k req/s) are measured beside it
                (extras), so the line carries every figure of the metric.
  large-arrays  16 fp64 arrays of 2^25 elements, each sent 4 times
                (64 transfers of 256 MiB); one digest launch per transfer;
                the metric is the digest rate in GB/s.
  trace         10^7 map records over 10^5 Zipf(1.1) slots plus kernel
                records; the analysis alone; metric in events/s.
  plain-small   64 buffers of 4 KiB-256 KiB and a 1,000-record log, digests
                by per-buffer launches (cache-resident, not an HBM figure).
  serve         open-loop Poisson arrivals at 10k, 50k and 200k requests/s,
                each a mapping record with a payload of log-uniform
                4 KiB-64 MiB from a 16 GiB device arena; continuous batching
                against the plain one-request-per-launch server; p50/p99
                latency (completion seen on the host - scheduled arrival).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch",
                    choices=["large-arrays", "batch", "trace", "plain-small", "serve", "rate-vs-size"])
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="serve: schedule length per rate (at most 200,000 requests)")
    ap.add_argument("--plain-requests", type=int, default=20_000,
                    help="serve: requests of each schedule replayed through the plain server")
    ap.add_argument("--cpu-seconds", type=float, default=6.0,
                    help="wall time of the oracle baseline sample (split between its one-thread and "
                         "all-thread legs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="batch: skip the per-buffer form and the large-arrays extras")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--blocks-per-cu", type=int, default=None, help="batched digest tuning override")
    ap.add_argument("--split-bytes", type=int, default=None, help="batched digest tuning override")
    ap.add_argument("--chunk-nodes", type=int, default=None, help="batched digest tuning override")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="apply a tuning file written by paper_2601_12713_amd/autotune.py")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="before the workload, one elementwise copy kernel (torch.neg on int32) reading and "
                         "writing BYTES: the calibration dispatch of the HBM byte counters")
    return ap.parse_args()


def traffic_from_profile(name, sources):
    """HBM bytes per launch of kernel `name` from its committed counter summary
    (profiles/<name>.pmc.txt), or None when the summary is missing or was taken
    on sources other than the current ones."""
    import hashlib
    path = os.path.join(HERE, "profiles", name + ".pmc.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(HERE, src), "rb") as f:
            h.update(f.read())
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != h.hexdigest():
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


DIGEST_SOURCES = ["paper_2601_12713_amd/csrc/digest.hip", "paper_2601_12713_amd/csrc/xxh64_dev.h",
                  "paper_2601_12713_amd/csrc/internal.h"]
ANALYSIS_SOURCES = ["paper_2601_12713_amd/csrc/analyze.hip", "paper_2601_12713_amd/csrc/internal.h"]


def host_info():
    cores = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


class KernelTimer:
    """HIP-event pairs around launches on a given stream; average duration."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e

    def stop(self, e0):
        e1 = self.torch.cuda.Event(enable_timing=True)
        e1.record(self.stream)
        self.pairs.append((e0, e1))

    def durations_ms(self):
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.pairs]

    def mean_ms(self):
        d = self.durations_ms()
        return float(np.mean(d)) if d else None

    def summary(self):
        """Mean, median, p10 and p90 of the timed durations (ms)."""
        d = self.durations_ms()
        if not d:
            return None
        return {"mean": round(float(np.mean(d)), 5), "median": round(float(np.median(d)), 5),
                "p10": round(float(np.percentile(d, 10)), 5), "p90": round(float(np.percentile(d, 90)), 5),
                "n": len(d)}


def timed_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step("timed")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / steps


# ---------------------------------------------------------------------------
def run_large_arrays(args, torch, odp, W):
    la = W.LargeArrays(seed=2, device="cuda")
    la.materialize()  # every transfer reads its own 256 MiB
    n = len(la.snapshots)
    nbytes = la.n_elem * 8
    ptrs = [s.data_ptr() for s in la.snapshots]
    sizes = [nbytes] * n
    stream = torch.cuda.current_stream()
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    ev = la.events.copy()
    d_ev = torch.from_numpy(ev.view(np.uint8).reshape(-1).copy()).to("cuda")
    ev_u64 = d_ev.view(torch.int64).view(n, 8)
    d_flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    timer = KernelTimer(torch, stream)

    def step(mode):
        # one call: the library launches the digest kernel once per buffer
        e0 = timer.start() if mode else None
        odp.digest_buffers_plain(ptrs, sizes, out, stream)
        if mode:
            timer.stop(e0)
        ev_u64[:, 0].copy_(out)  # digest field of each record
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=n)

    ms = timed_steps(torch, step, args.steps, args.warmup)
    rep = odp.report_to_dict(d_rep.cpu().numpy())
    kern_ms = timer.mean_ms() / n  # average over the n back-to-back launches
    total = n * nbytes
    value = total / (ms * 1e-3) / 1e9
    achieved = nbytes / (kern_ms * 1e-3) / 1e9
    # batched form of the same 64 buffers, for the batched-vs-per-buffer view
    dptr = torch.tensor(np.array(ptrs, dtype=np.uint64).view(np.int64), device="cuda")
    dsz = torch.tensor(np.array(sizes, dtype=np.uint64).view(np.int64), device="cuda")
    out_b = torch.zeros(n, dtype=torch.int64, device="cuda")
    btimer = KernelTimer(torch, stream)

    def bstep(mode):
        e0 = btimer.start() if mode else None
        odp.digest_buffers(dptr, dsz, out_b, stream)
        if mode:
            btimer.stop(e0)

    timed_steps(torch, bstep, args.steps, args.warmup)
    b_ms = btimer.mean_ms()
    assert torch.equal(out, out_b), "batched and per-buffer digests differ"
    assert rep["dd_events"] == la.planted_dd, (rep["dd_events"], la.planted_dd)
    line = {
        "metric": "digest GB/s (per-buffer launch, 256 MiB fp64 transfers) incl. trace analysis",
        "value": round(value, 1),
        "unit": "GB/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": "large-arrays: 16 fp64 arrays x 2^25 elements, each sent 4 times (64 x 256 MiB H2D "
                               "records), per-buffer digest launch, then analysis of the 64-record log",
                   "buffers": n, "bytes_per_step": total, "events": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("digest_one_kernel.large-arrays", DIGEST_SOURCES),
                     "kernel": "digest_one_kernel (one launch per 256 MiB buffer; HIP events around the 64 "
                               "back-to-back launches of a step, divided by 64)",
                     "kernel_ms": round(kern_ms, 5)},
        "extras": {"step_kernels_ms": timer.summary(),
                   "batched_GBps": round(total / (b_ms * 1e-3) / 1e9, 1),
                   "batched_frac_of_peak": round(total / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "per_buffer_GBps": round(achieved, 1),
                   "dd_events": rep["dd_events"], "planted_dd": la.planted_dd},
    }

    def cpu_sample(budget_s):
        host = [la.snapshots[i].cpu().numpy().view(np.uint8) for i in range(min(16, n))]
        one, many, T = oracle_rates(host, budget_s)
        return {"value": round(many, 3), "cores": T, "value_1_thread": round(one, 3),
                "sample": "the oracle (g++ -O3 -march=native on this host) digesting %d of the 256 MiB fp64 "
                          "arrays over and over: %.1f s on 1 thread, then %.1f s on %d threads over disjoint "
                          "arrays" % (len(host), budget_s / 2, budget_s / 2, T)}

    return line, cpu_sample


def oracle_threads():
    """Threads of the oracle's parallel leg: the host's cores, at most 16 (a
    one-GPU machine's share)."""
    return max(1, min(16, os.cpu_count() or 1))


def oracle_rates(host, budget_s):
    """Digest rate of the serial oracle over a list of host byte arrays: one
    thread for half the budget, then T threads over disjoint buffers (each
    thread walks its own share in turn) for the other half. The oracle is
    compiled for this host (-O3 -march=native) first, outside the timing."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.use_native_build(tempfile.mkdtemp(prefix="odp_oracle_"))
    done, k, t0 = 0, 0, time.perf_counter()
    while True:
        h = host[k % len(host)]
        oracle.d64(h)
        done += h.size
        k += 1
        if time.perf_counter() - t0 >= budget_s / 2:
            break
    one = done / (time.perf_counter() - t0) / 1e9
    T = oracle_threads()
    deadline = time.perf_counter() + budget_s / 2

    def worker(t):
        mine = host[t::T] or host[:1]
        got, j = 0, 0
        while time.perf_counter() < deadline:
            h = mine[j % len(mine)]
            oracle.d64(h)  # releases the GIL
            got += h.size
            j += 1
        return got

    t1 = time.perf_counter()
    with ThreadPoolExecutor(T) as ex:
        total = sum(ex.map(worker, range(T)))
    many = total / (time.perf_counter() - t1) / 1e9
    return one, many, T


def measure_large_arrays(torch, odp, W, steps):
    """The large-arrays workload's digest rates: per-buffer launches (HIP events
    around each step's 64 launches) and the batched form over the same buffers."""
    la = W.LargeArrays(seed=2, device="cuda")
    la.materialize()
    n = len(la.snapshots)
    nbytes = la.n_elem * 8
    ptrs = [s.data_ptr() for s in la.snapshots]
    sizes = [nbytes] * n
    stream = torch.cuda.current_stream()
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    timer = KernelTimer(torch, stream)

    def step(mode):
        e0 = timer.start() if mode else None
        odp.digest_buffers_plain(ptrs, sizes, out, stream)
        if mode:
            timer.stop(e0)

    timed_steps(torch, step, steps, 2)
    per = timer.summary()
    dptr = torch.tensor(np.array(ptrs, dtype=np.uint64).view(np.int64), device="cuda")
    dsz = torch.tensor(np.array(sizes, dtype=np.uint64).view(np.int64), device="cuda")
    out_b = torch.zeros(n, dtype=torch.int64, device="cuda")
    btimer = KernelTimer(torch, stream)

    def bstep(mode):
        e0 = btimer.start() if mode else None
        odp.digest_buffers(dptr, dsz, out_b, stream)
        if mode:
            btimer.stop(e0)

    timed_steps(torch, bstep, steps, 2)
    assert torch.equal(out, out_b), "batched and per-buffer digests differ"
    bsum = btimer.summary()
    total = n * nbytes
    res = {"buffers": n, "bytes": total,
           "per_buffer_GBps": round(total / (per["mean"] * 1e-3) / 1e9, 1),
           "per_buffer_kernel_us_mean": round(per["mean"] * 1e3 / n, 2),
           "per_buffer_kernel_us_median": round(per["median"] * 1e3 / n, 2),
           "per_buffer_frac_of_peak": round(total / (per["mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "batched_GBps": round(total / (bsum["mean"] * 1e-3) / 1e9, 1),
           "batched_frac_of_peak": round(total / (bsum["mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del la, out, out_b
    torch.cuda.empty_cache()
    return res


def run_batch(args, torch, odp, W):
    bb = W.BatchBuffers(seed=3, device="cuda")
    n = bb.sizes.size
    stream = torch.cuda.current_stream()
    dptr = torch.tensor(bb.pointers().view(np.int64), device="cuda")
    dsz = torch.tensor(bb.sizes.view(np.int64), device="cuda")
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    ev, tx = bb.transfer_log()
    m = len(ev)
    odp.reserve(max_buffers=n, max_total_bytes=int(bb.total_bytes), max_events=m, stream=stream)
    d_ev = torch.from_numpy(ev.view(np.uint8).reshape(-1).copy()).to("cuda")
    ev_u64 = d_ev.view(torch.int64).view(m, 8)
    d_tx = torch.from_numpy(tx.astype(np.int64)).to("cuda")
    d_flags = torch.zeros(m, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    dtimer = KernelTimer(torch, stream)
    atimer = KernelTimer(torch, stream)

    def step(mode):
        e0 = dtimer.start() if mode else None
        odp.digest_buffers(dptr, dsz, out, stream)  # plan + persistent digest + tree kernels, one graph
        if mode:
            dtimer.stop(e0)
        ev_u64[:, 0].index_copy_(0, d_tx, out)  # digest field of each transfer record
        e1 = atimer.start() if mode else None
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=m)
        if mode:
            atimer.stop(e1)

    ms = timed_steps(torch, step, args.steps, args.warmup)
    assert odp.device_status() == odp.ODP_OK
    dsum, asum = dtimer.summary(), atimer.summary()
    rep = odp.report_to_dict(d_rep.cpu().numpy())
    copies = int((bb.copy_of >= 0).sum())
    assert rep["dd_events"] == copies, (rep["dd_events"], copies)
    g = out.cpu().numpy()
    cp = bb.copy_of >= 0
    assert (g[cp] == g[bb.copy_of[cp]]).all(), "copies must digest like their sources"
    total = bb.total_bytes
    value = total / (ms * 1e-3) / 1e9
    achieved = total / (dsum["mean"] * 1e-3) / 1e9
    extras = {"tuning": odp.get_tuning(), "digest_ms": dsum, "analysis_ms": asum,
              "analysis_events_per_s": round(m / (asum["mean"] * 1e-3), 0),
              "digest_frac_of_peak_median": round(total / (dsum["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
              "dd_events": rep["dd_events"], "copies": copies, "ut_events": rep["ut_events"]}
    if not args.no_extras:
        hp, hs = bb.pointers().tolist(), bb.sizes.tolist()
        out_p = torch.zeros(n, dtype=torch.int64, device="cuda")
        ptimer = KernelTimer(torch, stream)

        def pstep(mode):
            e0 = ptimer.start() if mode else None
            odp.digest_buffers_plain(hp, hs, out_p, stream)
            if mode:
                ptimer.stop(e0)

        timed_steps(torch, pstep, 2, 1)
        p_ms = ptimer.mean_ms()
        assert torch.equal(out, out_p), "batched and per-buffer digests differ"
        extras.update({"per_buffer_GBps": round(total / (p_ms * 1e-3) / 1e9, 2), "per_buffer_ms": round(p_ms, 2),
                       "batched_vs_per_buffer": round(p_ms / dsum["mean"], 1)})
        del out_p
    line = {
        "metric": "batched digest GB/s, 100,000 buffers in one hipGraph-replayed launch (incl. trace analysis)",
        "value": round(value, 1),
        "unit": "GB/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": "batch: 100,000 buffers, log-uniform 64 B-16 MiB scaled to 48e9 bytes, "
                               "uint8/fp32/fp64 contents, 25%% copies; batched digest, then analysis of the "
                               "%d-record transfer log" % m,
                   "buffers": int(n), "bytes_per_step": int(total), "events": m},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("digest_batched_kernel.batch", DIGEST_SOURCES),
                     "kernel": "batched digest: one graph replay per step (plan kernels, digest_batched_kernel, "
                               "digest_tree_kernel); HIP events around the replay on the launch stream; "
                               "algorithmic bytes = the 48e9 bytes of the buffers",
                     "kernel_ms": dsum["mean"]},
        "extras": extras,
    }

    # the oracle baseline's sample: random whole buffers (~2 GB) copied to the host
    # now, outside any timing, so the device arena can be freed for the extras
    sample = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(0)
        pick, tot = [], 0
        for i in rng.permutation(n):
            pick.append(int(i))
            tot += int(bb.sizes[i])
            if tot >= 2e9:
                break
        sample = ([bb.buffer(i).cpu().numpy() for i in pick], tot)

    def cpu_sample(budget_s):
        host, tot = sample
        one, many, T = oracle_rates(host, budget_s)
        return {"value": round(many, 3), "cores": T, "value_1_thread": round(one, 3),
                "sample": "the oracle (g++ -O3 -march=native on this host) digesting %d random buffers of the batch "
                          "(%.2f GB, host copies made before timing) over and over: %.1f s on 1 thread, then "
                          "%.1f s on %d threads over disjoint buffers" % (len(host), tot / 1e9, budget_s / 2,
                                                                          budget_s / 2, T)}

    if not args.no_extras:
        del bb, dptr, dsz, d_ev, ev_u64
        torch.cuda.empty_cache()
        extras["large_arrays"] = measure_large_arrays(torch, odp, W, max(5, args.steps))
        # the other two figures of the headline metric, so that this line carries them
        # too: the trace analysis (--workload trace) and serving latency (--workload
        # serve, here two rates over half a second each)
        extras["trace"] = measure_trace(torch, odp, W, max(5, args.steps))
        torch.cuda.empty_cache()
        rates, sb, _ = measure_serve(torch, odp, W, (50_000, 200_000), 0.5, steps=1, warmup=1)
        extras["serve"] = dict(rates, server_state_bytes=sb)
    return line, (cpu_sample if sample else None)


def run_rate_vs_size(args, torch, odp, W):
    """Per-buffer digest rate against buffer size, beside the host<->device copy
    rates of the same sizes (pinned host memory, one copy per call): whether
    fingerprinting a transfer on the device costs less than the transfer."""
    sizes = [1, 64, 4096, 1 << 16, 1 << 20, 1 << 24, 1 << 28, 1 << 30]
    big = sizes[-1]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    dev = torch.randint(0, 256, (big,), dtype=torch.uint8, device="cuda", generator=gen)
    host = torch.empty(big, dtype=torch.uint8, pin_memory=True)
    stream = torch.cuda.current_stream()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ptr = dev.data_ptr()

    def per_call_us(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / reps

    # Digest launches replayed from a graph give the device time per launch
    # without the host's submission cost. The first call on the capture stream
    # (largest size) sets up that stream's workspace outside any capture.
    cap = torch.cuda.Stream()
    with torch.cuda.stream(cap):
        odp.digest_buffers_plain([ptr], [big], out, cap)
    cap.synchronize()

    def graph_us(sz, reps):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cap):
            for _ in range(reps):
                odp.digest_buffers_plain([ptr], [sz], out, cap)
        g.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / reps

    rows = {}
    t0 = time.perf_counter()
    for sz in sizes:
        reps = max(5, min(400, (1 << 31) // (sz * 4) if sz >= 4096 else 400))
        k_us = graph_us(sz, min(200, reps))
        d_us = per_call_us(lambda: odp.digest_buffers_plain([ptr], [sz], out, stream), reps)
        h_us = per_call_us(lambda: dev[:sz].copy_(host[:sz], non_blocking=True), reps)
        g_us = per_call_us(lambda: host[:sz].copy_(dev[:sz], non_blocking=True), reps)
        rows[str(sz)] = {"digest_us": round(d_us, 2), "digest_GBps": round(sz / d_us / 1e3, 3),
                         "digest_graph_us": round(k_us, 2),
                         "h2d_us": round(h_us, 2), "h2d_GBps": round(sz / h_us / 1e3, 3),
                         "d2h_us": round(g_us, 2), "d2h_GBps": round(sz / g_us / 1e3, 3),
                         "digest_vs_h2d": round(h_us / d_us, 2)}
    wall_ms = (time.perf_counter() - t0) * 1000.0
    top = rows[str(big)]
    achieved = top["digest_GBps"]
    line = {
        "metric": "per-buffer digest GB/s at 1 GiB (digest and copy rates by size in extras)",
        "value": achieved,
        "unit": "GB/s",
        "ms_per_step": round(wall_ms, 3),
        "config": {"workload": "rate-vs-size: one buffer of 1 B-1 GiB per call, digest vs pinned H2D/D2H copy",
                   "sizes": sizes},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "digest_one_kernel, one launch over 1 GiB (HIP events per call)",
                     "kernel_ms": round(top["digest_us"] / 1000.0, 4)},
        "extras": rows,
    }
    return line, None


def measure_trace(torch, odp, W, steps):
    """The trace workload's analysis timed with HIP events (planted counts checked)."""
    tr = W.TraceAtScale(seed=4)
    n = len(tr.events)
    stream = torch.cuda.current_stream()
    d_ev = torch.from_numpy(tr.events.view(np.uint8).reshape(-1).copy()).to("cuda")
    d_flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    odp.reserve(max_events=n, stream=stream)
    timer = KernelTimer(torch, stream)

    def step(mode):
        e0 = timer.start() if mode else None
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=n)
        if mode:
            timer.stop(e0)

    timed_steps(torch, step, steps, 2)
    rep = odp.report_to_dict(d_rep.cpu().numpy())
    for k, v in tr.planted.items():
        assert rep[k] == v, (k, rep[k], v)
    t = timer.summary()
    return {"events": n, "ms": t, "events_per_s": round(n / (t["median"] * 1e-3), 0),
            "frac_of_peak_65B_per_record": round(65.0 * n / (t["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_trace(args, torch, odp, W):
    tr = W.TraceAtScale(seed=4)
    n = len(tr.events)
    stream = torch.cuda.current_stream()
    d_ev = torch.from_numpy(tr.events.view(np.uint8).reshape(-1).copy()).to("cuda")
    d_flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    odp.reserve(max_events=n, stream=stream)
    timer = KernelTimer(torch, stream)

    def step(mode):
        e0 = timer.start() if mode else None
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=n)
        if mode:
            timer.stop(e0)

    ms = timed_steps(torch, step, args.steps, args.warmup)
    rep = odp.report_to_dict(d_rep.cpu().numpy())
    for k, v in tr.planted.items():
        assert rep[k] == v, (k, rep[k], v)
    kern_ms = timer.mean_ms()
    value = n / (ms * 1e-3)
    alg_bytes = 65.0 * n
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    line = {
        "metric": "trace analysis events/s",
        "value": round(value, 0),
        "unit": "events/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": "trace: 10^7 map records over 10^5 Zipf(1.1) slots + kernel records", "events": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("analysis.trace", ANALYSIS_SOURCES),
                     "kernel": "whole analysis (65 algorithmic bytes per record; traffic: HBM bytes of all its "
                               "kernels per call)", "kernel_ms": round(kern_ms, 4)},
        "extras": {k: rep[k] for k in ("dd_events", "rt_pairs", "ra_events", "ua_events")},
    }
    if line["roofline"]["traffic"]:
        line["extras"]["measured_GBps"] = round(line["roofline"]["traffic"] / (kern_ms * 1e-3) / 1e9, 1)

    def cpu_sample(budget_s):
        import tempfile
        import oracle
        oracle.use_native_build(tempfile.mkdtemp(prefix="odp_oracle_"))
        m = 1
        while True:
            sub = tr.events[:m]
            t0 = time.perf_counter()
            oracle.analyze(sub)
            el = time.perf_counter() - t0
            if el * 4 >= budget_s or m >= n:
                return {"value": round(m / el, 0), "cores": 1,
                        "sample": "the oracle (g++ -O3 -march=native on this host, one thread: its rules are "
                                  "chronological passes) on the first %d records (%.1f s)" % (m, el)}
            m = min(n, m * 4)

    return line, cpu_sample


def run_plain_small(args, torch, odp, W):
    ps = W.PlainSmall(seed=1)
    stream = torch.cuda.current_stream()
    snaps = [torch.from_numpy(s).to("cuda") for s in ps.snapshots]
    tx = np.nonzero(ps.snapshot_of >= 0)[0]
    ptrs = [snaps[ps.snapshot_of[i]].data_ptr() for i in tx]
    sizes = [ps.snapshots[ps.snapshot_of[i]].size for i in tx]
    n = len(ps.events)
    out = torch.zeros(len(tx), dtype=torch.int64, device="cuda")
    d_ev = torch.from_numpy(ps.events.view(np.uint8).reshape(-1).copy()).to("cuda")
    ev_u64 = d_ev.view(torch.int64).view(n, 8)
    d_tx = torch.from_numpy(tx.astype(np.int64)).to("cuda")
    d_flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")

    def step(mode):
        odp.digest_buffers_plain(ptrs, sizes, out, stream)
        ev_u64[:, 0].index_copy_(0, d_tx, out)
        odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=n)

    ms = timed_steps(torch, step, args.steps, args.warmup)
    total = int(np.sum(sizes))
    line = {
        "metric": "digest + flags per step (per-buffer launches; cache-resident)",
        "value": round(n / (ms * 1e-3), 0),
        "unit": "events/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": "plain-small: 64 buffers 4 KiB-256 KiB, 1,000-record log", "events": n,
                   "transfers": int(len(tx)), "bytes_digested": total},
        "roofline": None,
        "extras": {"digest_GBps_cache_resident": round(total / (ms * 1e-3) / 1e9, 2)},
    }
    return line, None


def measure_serve(torch, odp, W, rate_list, seconds, steps, warmup, plain_requests=0, burst=False):
    """Serving schedules at the given rates (batched server; the plain one too when
    plain_requests > 0; the 64 MiB burst when burst): p50/p99 latency and GB/s per rate."""
    gib = 1 << 30
    arena = torch.empty(16 * gib, dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for off in range(0, arena.numel(), gib):
        arena[off:off + gib].copy_(torch.randint(0, 256, (gib,), dtype=torch.uint8, device="cuda", generator=gen))
    torch.cuda.synchronize()
    budget = 32 * 10**9  # device memory: the server's state and workspace plus the payloads in flight

    def serve(sched, mode, n):
        srv = odp.Server(max_events=n, budget_bytes=budget, mode=mode)
        done, st = srv.run(sched.events[:n], sched.payload_ptrs()[:n], sched.payload_bytes[:n], sched.arrival_ns[:n])
        srv.close()
        state_bytes[0] = max(state_bytes[0], st["state_bytes"])
        lat_us = (done.astype(np.float64) - sched.arrival_ns[:n].astype(np.float64)) / 1e3
        return {"requests": n, "p50_us": round(float(np.percentile(lat_us, 50)), 1),
                "p99_us": round(float(np.percentile(lat_us, 99)), 1), "GBps": round(st["bytes"] / st["seconds"] / 1e9, 1),
                "offered_GBps": (round(float(sched.payload_bytes[:n].sum()) / float(sched.arrival_ns[n - 1]), 1)
                                 if sched.arrival_ns[n - 1] else None),
                "seconds": round(st["seconds"], 3), "ticks": st["ticks"], "max_tick": st["max_tick"],
                "budget_waits": st["budget_waits"]}

    state_bytes = [0]
    warm = W.ServingSchedule(seed=100, n=2000, rate=50_000.0, arena=arena)
    for _ in range(max(warmup, 1)):
        serve(warm, odp.SERVER_BATCHED, 2000)
        if plain_requests:
            serve(warm, odp.SERVER_PLAIN, 500)
    rates = {}
    t0 = time.perf_counter()
    for rate in rate_list:
        n = int(min(200_000, rate * seconds))
        sched = W.ServingSchedule(seed=6, n=n, rate=float(rate), arena=arena)
        runs = [serve(sched, odp.SERVER_BATCHED, n) for _ in range(steps)]
        r = max(runs, key=lambda x: x["p99_us"])  # the worst of the repeats
        if plain_requests:
            r["plain"] = serve(sched, odp.SERVER_PLAIN, min(n, plain_requests))
        rates["%dk_per_s" % (rate // 1000)] = r
    ms = (time.perf_counter() - t0) * 1e3 / (len(rate_list) * steps)
    if burst:
        # 1000 requests of 64 MiB at t = 0 against the same budget
        b = W.ServingSchedule(seed=7, n=1000, rate=1e9, lo=64 << 20, hi=64 << 20, arena=arena)
        b.arrival_ns[:] = 0
        rates["burst_1000x64MiB"] = serve(b, odp.SERVER_BATCHED, 1000)
    del arena
    torch.cuda.empty_cache()
    return rates, state_bytes[0], ms


def run_serve(args, torch, odp, W):
    rates, state_bytes, ms = measure_serve(torch, odp, W, (10_000, 50_000, 200_000), args.serve_seconds, args.steps,
                                           args.warmup, plain_requests=args.plain_requests, burst=True)
    top = rates["200k_per_s"]
    line = {
        "metric": "serving GB/s at 200k req/s (p50/p99 latency in extras)",
        "value": top["GBps"],
        "unit": "GB/s",
        "ms_per_step": round(ms, 3),
        "config": {"workload": "serve: Poisson 10k/50k/200k req/s, payloads log-uniform 4 KiB-64 MiB of a 16 GiB "
                               "arena, 20% repeats, planted round trips; 32e9-byte device memory budget (the "
                               "server's state and workspace plus the payloads in flight)",
                   "server_state_bytes": state_bytes,
                   "requests_per_rate": [v["requests"] for k, v in rates.items() if k.endswith("_per_s")]},
        "roofline": None,
        "extras": rates,
    }
    return line, None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported (the multi-GPU split of the work "
              "is not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2601_12713_amd import odp
    from paper_2601_12713_amd import workloads as W
    odp.load()
    if args.tuning:
        from paper_2601_12713_amd import autotune
        autotune.apply(args.tuning)
    if args.blocks_per_cu is not None or args.split_bytes is not None or args.chunk_nodes is not None:
        odp.set_tuning(blocks_per_cu=args.blocks_per_cu, split_bytes=args.split_bytes, chunk_nodes=args.chunk_nodes)
    if args.copy_probe:
        src = torch.randint(0, 1 << 30, (args.copy_probe // 4,), dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    runner = {"large-arrays": run_large_arrays, "batch": run_batch, "trace": run_trace,
              "plain-small": run_plain_small, "serve": run_serve, "rate-vs-size": run_rate_vs_size}[args.workload]
    line, cpu_sample = runner(args, torch, odp, W)
    out = {"metric": line["metric"], "value": line["value"], "unit": line["unit"], "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": line["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic (seeded; shapes of the paper's workloads)", "config": line["config"],
           "roofline": line["roofline"]}
    if cpu_sample is not None and not args.no_cpu_baseline:
        cb = cpu_sample(args.cpu_seconds)
        cores, model = host_info()
        out["cpu_baseline"] = {"value": cb.pop("value"), "unit": line["unit"], "cores": cb.pop("cores"),
                               "kind": "oracle", "sample": cb.pop("sample"), **cb,
                               "host_cores": cores, "host_cpu": model}
    out["extras"] = line.get("extras")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
