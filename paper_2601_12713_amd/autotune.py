"""Autotuner of the batched digest's launch parameters.

Searches workgroups per compute unit x the one-wavefront split (the size of a
level-1 node below which one wavefront, not a whole workgroup, hashes it) x the
chunk (work items a workgroup claims at once: 1-8 level-1 nodes, 64-512
consecutive leaves) on a held-out batch (seed 101, the batch workload's size distribution at a smaller
total), times each point with HIP events on the launch stream, checks that
every point returns the same digests, and writes a per-device JSON. The leaf
(4096 B) and fan-in (64) belong to the digest definition and are not tuned.

    python -m paper_2601_12713_amd.autotune [--out PATH] [--total-bytes B] [--buffers N]

`apply(path)` loads such a file into the library (odp_set_tuning); the
binding applies `tuning/<arch>.json` next to this file when it exists.
"""
import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BLOCKS_PER_CU = (1, 2, 4, 8)
SPLITS = (0, 16384, 32768, 65536)
CHUNKS = (1, 2, 4, 8)


def default_path(arch):
    return os.path.join(HERE, "tuning", "%s.json" % arch)


def apply(path):
    from . import odp
    with open(path) as f:
        best = json.load(f)["best"]
    odp.set_tuning(blocks_per_cu=int(best["blocks_per_cu"]), split_bytes=int(best["split_bytes"]),
                   chunk_nodes=int(best.get("chunk_nodes", 1)), use_graph=1)
    return best


def tune(total_bytes=8_000_000_000, n=20_000, reps=5, warmup=2, log=print):
    import torch

    from . import odp
    from . import workloads as W
    odp.load()
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    bb = W.BatchBuffers(seed=101, n=n, cap_total=total_bytes, device="cuda")
    stream = torch.cuda.current_stream()
    dptr = torch.tensor(bb.pointers().view(np.int64), device="cuda")
    dsz = torch.tensor(bb.sizes.view(np.int64), device="cuda")
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    odp.reserve(max_buffers=n, max_total_bytes=int(bb.total_bytes), stream=stream)
    saved = odp.get_tuning()
    points, ref = [], None
    try:
        for bpc, split, chunk in [(b, s, c) for b in BLOCKS_PER_CU for s in SPLITS for c in CHUNKS]:
            odp.set_tuning(blocks_per_cu=bpc, split_bytes=split, chunk_nodes=chunk, use_graph=1)
            for _ in range(warmup):
                odp.digest_buffers(dptr, dsz, out, stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                odp.digest_buffers(dptr, dsz, out, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            got = out.cpu().numpy()
            if ref is None:
                ref = got.copy()
            if not np.array_equal(got, ref):
                raise RuntimeError("tuning point %s gave different digests" % ((bpc, split, chunk),))
            gbps = bb.total_bytes / (ms * 1e-3) / 1e9
            points.append({"blocks_per_cu": bpc, "split_bytes": split, "chunk_nodes": chunk, "ms": round(ms, 4),
                           "GBps": round(gbps, 1)})
            log("blocks_per_cu=%d split_bytes=%6d chunk_nodes=%d  %.3f ms  %.1f GB/s" % (bpc, split, chunk, ms, gbps))
    finally:
        odp.set_tuning(**saved)
    best = max(points, key=lambda p: p["GBps"])
    return {
        "device": props.name, "arch": arch, "compute_units": props.multi_processor_count,
        "workload": "held-out batch: seed 101, %d buffers, log-uniform 64 B-16 MiB scaled to %d bytes" % (
            n, int(bb.total_bytes)),
        "reps": reps, "timed_with": "HIP events on the launch stream around %d graph replays" % reps,
        "created": time.strftime("%Y-%m-%d %H:%M:%S"), "points": points,
        "best": {"blocks_per_cu": best["blocks_per_cu"], "split_bytes": best["split_bytes"],
                 "chunk_nodes": best["chunk_nodes"], "use_graph": 1},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--total-bytes", type=int, default=8_000_000_000)
    ap.add_argument("--buffers", type=int, default=20_000)
    args = ap.parse_args()
    res = tune(total_bytes=args.total_bytes, n=args.buffers)
    path = args.out or default_path(res["arch"])
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["best"]))
    print("wrote", path)


if __name__ == "__main__":
    main()
