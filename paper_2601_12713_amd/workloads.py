"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no part of the method: it draws buffers, event logs and
arrival schedules from seeds and records what it planted, and both the GPU path
and the CPU oracle consume what it returns. It never computes a digest or a
flag; a transfer's ``digest`` field is left 0 where the digest must come from
the bytes (each side fills it in from the same bytes), and is drawn at random
where the workload specifies digests directly (the trace-at-scale log).

Shapes follow the paper's applications as described in its evaluation
(Sec. 7.2, App. C): large fp64 arrays re-sent every iteration (babelstream),
tiny scalars and structs next to large arrays, and duplicate / round-trip /
repeated / unused mixes of the magnitudes in the issue table (Sec. 7.5).
"""
import math

import numpy as np

# The 64-byte event record of include/odp.h.
EVENT_DTYPE = np.dtype([
    ("digest", "<u8"), ("src_addr", "<u8"), ("dst_addr", "<u8"), ("bytes", "<u8"),
    ("t_start", "<u8"), ("t_end", "<u8"), ("codeptr", "<u8"),
    ("src_dev", "<i2"), ("dst_dev", "<i2"), ("op", "u1"), ("rsv0", "u1"), ("rsv1", "<u2"),
])
assert EVENT_DTYPE.itemsize == 64

ALLOC, H2D, D2H, D2D, DELETE, KERNEL = 1, 2, 3, 4, 5, 6
HOST = -1
HOST_BASE = 0x7F00_0000_0000
DEV_BASE = 0x7E00_0000_0000


def empty_events(n):
    return np.zeros(n, dtype=EVENT_DTYPE)


def _times(rng, n, nbytes, gap_ns=1000.0, base_ns=5000, rate_bytes_per_ns=25.0):
    """Disjoint, increasing intervals: gap ~ Exp(gap_ns) (at least 1 ns), duration = base + bytes/rate."""
    gaps = np.maximum(1, rng.exponential(gap_ns, size=n)).astype(np.uint64)
    durs = (base_ns + np.asarray(nbytes, dtype=np.float64) / rate_bytes_per_ns).astype(np.uint64)
    t_start = np.empty(n, dtype=np.uint64)
    t_end = np.empty(n, dtype=np.uint64)
    step = gaps + durs
    ends = np.cumsum(step, dtype=np.uint64)
    t_end[:] = ends
    t_start[:] = ends - durs
    return t_start, t_end


# ----------------------------------------------------------------------------
# Tiny random traces with real byte payloads (for brute-force checks).
# ----------------------------------------------------------------------------
def tiny_trace(seed, n_events=40, n_devices=1, n_payloads=6, n_vars=4, invalid_rate=0.0,
               max_payload=300, overlap_kernels=False):
    """A short random log over host + ``n_devices`` devices.

    Returns (events, payloads, payload_of): ``payloads`` is a list of byte
    strings (some byte-identical on purpose), ``payload_of[i]`` the payload a
    transfer i carries (-1 for other records). Digest fields are left 0.
    """
    rng = np.random.default_rng(seed)
    payloads = []
    for k in range(n_payloads):
        if k > 0 and rng.random() < 0.3:
            payloads.append(bytes(payloads[int(rng.integers(0, k))]))  # equal bytes, separate object
        elif k > 0 and rng.random() < 0.2:
            src = bytearray(payloads[int(rng.integers(0, k))])
            if len(src) == 0:
                src = bytearray(b"\x00")
            src[int(rng.integers(0, len(src)))] ^= 1 << int(rng.integers(0, 8))  # one bit away
            payloads.append(bytes(src))
        else:
            ln = int(rng.integers(0, max_payload + 1))
            payloads.append(rng.integers(0, 256, size=ln, dtype=np.uint8).tobytes())
    ev = empty_events(n_events)
    payload_of = np.full(n_events, -1, dtype=np.int64)
    devs = list(range(n_devices))
    ops = rng.choice([ALLOC, H2D, D2H, D2D, DELETE, KERNEL], size=n_events,
                     p=[0.14, 0.3, 0.2, 0.08 if n_devices > 1 else 0.0, 0.14, 0.14 if n_devices > 1 else 0.22])
    t = 0
    for i in range(n_events):
        op = int(ops[i])
        if op == D2D and n_devices < 2:
            op = H2D
        ev["op"][i] = op
        gap = int(rng.integers(0, 3))  # ties in t_start occur on purpose
        t += gap
        ev["t_start"][i] = t
        if op == KERNEL and overlap_kernels:
            ev["t_end"][i] = t + int(rng.integers(0, 12))
        else:
            ev["t_end"][i] = t + int(rng.integers(0, 3))
        if op in (H2D, D2H, D2D):
            p = int(rng.integers(0, n_payloads))
            payload_of[i] = p
            ev["bytes"][i] = len(payloads[p])
            if op == H2D:
                s, d = HOST, int(rng.choice(devs))
            elif op == D2H:
                s, d = int(rng.choice(devs)), HOST
            else:
                s, d = int(rng.choice(devs)), int(rng.choice(devs))  # self-transfers occur
            ev["src_dev"][i], ev["dst_dev"][i] = s, d
            v = int(rng.integers(0, n_vars))
            ev["src_addr"][i] = HOST_BASE + v * 4096
            ev["dst_addr"][i] = DEV_BASE + v * 4096
        elif op in (ALLOC, DELETE):
            v = int(rng.integers(0, n_vars))
            ev["dst_dev"][i] = int(rng.choice(devs))
            ev["src_dev"][i] = HOST
            ev["src_addr"][i] = HOST_BASE + v * 4096
            ev["dst_addr"][i] = DEV_BASE + v * 4096
            ev["bytes"][i] = int(rng.choice([64, 128]))
        else:
            ev["dst_dev"][i] = int(rng.choice(devs))
            ev["src_dev"][i] = HOST
        ev["codeptr"][i] = 0x400000 + 16 * i
        if invalid_rate > 0 and rng.random() < invalid_rate:
            kind = int(rng.integers(0, 4))
            if kind == 0:
                ev["op"][i] = int(rng.choice([0, 7, 200]))
            elif kind == 1 and i > 0:
                ev["t_start"][i] = max(0, int(ev["t_start"][i - 1]) - 1 - int(rng.integers(0, 2)))
                ev["t_end"][i] = ev["t_start"][i]
            elif kind == 2:
                ev["t_end"][i] = ev["t_start"][i] - 1 if ev["t_start"][i] > 0 else 0
                if ev["t_start"][i] == 0:
                    ev["t_start"][i] = 1
            else:
                ev["dst_dev"][i] = int(rng.choice([-2, 10, 300]))
    return ev, payloads, payload_of


# ----------------------------------------------------------------------------
# Plain, small: 64 buffers and a 1,000-record log replayed over them.
# ----------------------------------------------------------------------------
class PlainSmall:
    """64 device-resident buffers (4 KiB-256 KiB, 30% byte copies of earlier ones)
    and a 1,000-record log on {host, device 0} that maps them in episodes.

    A KERNEL record mutates one resident buffer (XOR of one 8-byte word), so the
    content moved by a transfer is a *snapshot*: ``snapshots`` lists the
    distinct contents (numpy uint8 arrays) and ``snapshot_of[i]`` the snapshot
    transfer i carries. Planted: about 20% of host-to-device records re-send an
    unmodified buffer (duplicates) and about 5% of records are the host-to-device
    return of a buffer just copied back unmodified (round trips).
    ``planted_dd`` / ``planted_rt_rx`` / ``planted_rt_tx`` hold record indices.
    """

    def __init__(self, seed=1, n_buffers=64, n_events=1000, min_size=4096, max_size=262144, copy_frac=0.30):
        rng = np.random.default_rng(seed)
        sizes = rng.integers(min_size, max_size + 1, size=n_buffers)
        content = []
        n_copies = int(round(copy_frac * n_buffers))
        copy_idx = set(rng.choice(np.arange(1, n_buffers), size=n_copies, replace=False).tolist())
        self.copy_of = {}
        for b in range(n_buffers):
            if b in copy_idx:
                src = int(rng.integers(0, b))
                self.copy_of[b] = src
                content.append(content[src].copy())
                sizes[b] = content[src].size
            else:
                content.append(rng.integers(0, 256, size=int(sizes[b]), dtype=np.uint8))
        self.initial = [c.copy() for c in content]
        self.sizes = sizes.astype(np.uint64)
        version = [0] * n_buffers
        snap_id = {}
        content_id = {}  # exact bytes -> content number (byte-identical buffers share one)
        self.snapshots = []
        self.content_of_snapshot = []

        def snapshot(b):
            key = (b, version[b])
            if key not in snap_id:
                snap_id[key] = len(self.snapshots)
                self.snapshots.append(content[b].copy())
                self.content_of_snapshot.append(content_id.setdefault(content[b].tobytes(), len(content_id)))
            return snap_id[key]

        recs = []  # (op, buf, snapshot)
        resident = set()
        self.planted_dd, self.planted_rt_rx, self.planted_rt_tx = [], [], []
        dev_received = set()  # contents device 0 has received
        last_move = {}  # content -> (record index, op) of its latest transfer

        def emit(op, b):
            s = snapshot(b)
            c = self.content_of_snapshot[s]
            if op == H2D:
                dev_received.add(c)
            last_move[c] = (len(recs), op)
            recs.append((op, b, s))

        def current(b):
            return self.content_of_snapshot[snapshot(b)]

        while len(recs) < n_events:
            u = rng.random()
            free = [b for b in range(n_buffers) if b not in resident]
            res = sorted(resident)
            if (u < 0.20 or not res) and free:
                b = int(rng.choice(free))
                recs.append((ALLOC, b, -1))
                resident.add(b)
                emit(H2D, b)
            elif u < 0.40 and res:
                b = int(rng.choice(res))
                w = int(rng.integers(0, content[b].size // 8))
                mask = rng.integers(1, 2**63, size=1, dtype=np.int64).view(np.uint8)
                content[b][8 * w:8 * w + 8] ^= mask
                version[b] += 1
                recs.append((KERNEL, b, -1))
            elif u < 0.48 and res:
                # planted duplicate: re-send bytes device 0 already received
                cand = [b for b in res if current(b) in dev_received]
                if cand:
                    b = int(rng.choice(cand))
                    self.planted_dd.append(len(recs))
                    emit(H2D, b)
            elif u < 0.70 and res:
                emit(D2H, int(rng.choice(res)))
            elif u < 0.77 and res:
                # planted round trip: send back bytes whose latest move was device 0 -> host
                cand = [b for b in res if last_move.get(current(b), (0, 0))[1] == D2H]
                if cand:
                    b = int(rng.choice(cand))
                    self.planted_rt_tx.append(last_move[current(b)][0])
                    self.planted_rt_rx.append(len(recs))
                    emit(H2D, b)
            elif res:
                b = int(rng.choice(res))
                emit(D2H, b)
                recs.append((DELETE, b, -1))
                resident.discard(b)
        recs = recs[:n_events]
        # planted records beyond the cut are dropped
        n = len(recs)
        self.planted_dd = [i for i in self.planted_dd if i < n]
        keep = [(t, r) for t, r in zip(self.planted_rt_tx, self.planted_rt_rx) if r < n]
        self.planted_rt_tx = [t for t, _ in keep]
        self.planted_rt_rx = [r for _, r in keep]
        ev = empty_events(n)
        self.snapshot_of = np.full(n, -1, dtype=np.int64)
        nbytes = np.zeros(n, dtype=np.uint64)
        for i, (op, b, s) in enumerate(recs):
            ev["op"][i] = op
            ev["codeptr"][i] = 0x401000 + 32 * b
            if op == KERNEL:
                ev["dst_dev"][i], ev["src_dev"][i] = 0, HOST
                continue
            nbytes[i] = self.sizes[b]
            ev["bytes"][i] = self.sizes[b]
            if op in (ALLOC, DELETE):
                ev["src_dev"][i], ev["dst_dev"][i] = HOST, 0
                ev["src_addr"][i] = HOST_BASE + b * (1 << 20)
                ev["dst_addr"][i] = DEV_BASE + b * (1 << 20)
            elif op == H2D:
                ev["src_dev"][i], ev["dst_dev"][i] = HOST, 0
                ev["src_addr"][i] = HOST_BASE + b * (1 << 20)
                ev["dst_addr"][i] = DEV_BASE + b * (1 << 20)
                self.snapshot_of[i] = s
            else:
                ev["src_dev"][i], ev["dst_dev"][i] = 0, HOST
                ev["src_addr"][i] = DEV_BASE + b * (1 << 20)
                ev["dst_addr"][i] = HOST_BASE + b * (1 << 20)
                self.snapshot_of[i] = s
        ev["t_start"], ev["t_end"] = _times(rng, n, nbytes)
        self.events = ev


# ----------------------------------------------------------------------------
# Large arrays: 16 fp64 arrays of 2^25 elements, each sent 4 times.
# ----------------------------------------------------------------------------
class LargeArrays:
    """``n_arrays`` fp64 arrays of ``n_elem`` N(0,1) values, each sent once and
    re-sent ``resends`` times. Each re-send is, with probability 1/2, byte-identical
    to the array's current content; otherwise one element (never one flipped
    before in that array) has its lowest mantissa bit flipped first.

    Contents are drawn with torch on ``device`` (so large arrays never pass
    through host memory); ``snapshots`` is a list of torch float64 tensors in
    record order and ``planted_dd`` counts the byte-identical re-sends.
    """

    def __init__(self, seed=2, n_arrays=16, n_elem=1 << 25, resends=3, device="cpu"):
        import torch
        rng = np.random.default_rng(seed)
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        self.n_arrays, self.n_elem = n_arrays, n_elem
        current = [torch.randn(n_elem, dtype=torch.float64, device=device, generator=gen) for _ in range(n_arrays)]
        flipped = [set() for _ in range(n_arrays)]
        self.snapshots = []
        self.array_of = []
        self.identical = []
        self.planted_dd = 0
        for r in range(resends + 1):
            for a in range(n_arrays):
                if r > 0:
                    same = bool(rng.random() < 0.5)
                    if same:
                        self.planted_dd += 1
                    else:
                        while True:
                            e = int(rng.integers(0, n_elem))
                            if e not in flipped[a]:
                                break
                        flipped[a].add(e)
                        cur = current[a].clone()
                        cur.view(torch.int64)[e] ^= 1
                        current[a] = cur
                    self.identical.append(same)
                else:
                    self.identical.append(False)
                self.snapshots.append(current[a])  # shared tensor when identical
                self.array_of.append(a)
        n = len(self.snapshots)
        ev = empty_events(n)
        ev["op"] = H2D
        ev["src_dev"], ev["dst_dev"] = HOST, 0
        nbytes = np.full(n, n_elem * 8, dtype=np.uint64)
        ev["bytes"] = nbytes
        arr = np.array(self.array_of, dtype=np.uint64)
        ev["src_addr"] = np.uint64(HOST_BASE) + arr * np.uint64(1 << 30)
        ev["dst_addr"] = np.uint64(DEV_BASE) + arr * np.uint64(1 << 30)
        ev["codeptr"] = np.uint64(0x402000)
        ev["t_start"], ev["t_end"] = _times(rng, n, nbytes)
        self.events = ev

    def materialize(self):
        """Give every record its own copy (distinct HBM for every digest call)."""
        self.snapshots = [s.clone() for s in self.snapshots]


# ----------------------------------------------------------------------------
# Batching: many buffers of log-uniform sizes.
# ----------------------------------------------------------------------------
def batch_sizes(seed=3, n=100_000, lo=64, hi=1 << 24, cap_total=48_000_000_000):
    """Log-uniform sizes in [lo, hi], scaled down uniformly so the total stays
    under ``cap_total`` bytes, then rounded down to the element size of a dtype
    drawn uniformly from {uint8, float32, float64}. Returns (sizes u64, dtype codes u8: 0=u8, 1=f32, 2=f64)."""
    rng = np.random.default_rng(seed)
    raw = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)))
    total = raw.sum()
    if cap_total is not None and total > cap_total:
        raw = np.maximum(lo, np.floor(raw * (cap_total / total)))
    kinds = rng.integers(0, 3, size=n).astype(np.uint8)
    elem = np.array([1, 4, 8], dtype=np.float64)[kinds]
    sizes = (np.floor(raw / elem) * elem).astype(np.uint64)
    return sizes, kinds


class BatchBuffers:
    """``n`` buffers (sizes from ``batch_sizes``) laid out at 256-byte aligned
    offsets of one device arena; uint8 buffers hold uniform bytes, float32 and
    float64 buffers N(0,1) values; a fraction ``dup_frac`` are byte copies of an
    earlier buffer (same dtype class) at their own offsets.

    ``offsets`` / ``sizes`` describe the layout, ``copy_of[i]`` = source or -1.
    """

    def __init__(self, seed=3, n=100_000, lo=64, hi=1 << 24, cap_total=48_000_000_000, dup_frac=0.25,
                 device="cpu", align=256):
        import torch
        rng = np.random.default_rng(seed + 1000)
        sizes, kinds = batch_sizes(seed, n, lo, hi, cap_total)
        copy_of = np.full(n, -1, dtype=np.int64)
        dup = rng.random(n) < dup_frac
        dup[0] = False
        for i in np.nonzero(dup)[0]:
            j = int(rng.integers(0, i))
            while copy_of[j] >= 0:
                j = int(copy_of[j])
            copy_of[i] = j
            sizes[i] = sizes[j]
            kinds[i] = kinds[j]
        padded = ((sizes + np.uint64(align - 1)) // np.uint64(align)) * np.uint64(align)
        padded = np.maximum(padded, np.uint64(align))
        offsets = np.zeros(n, dtype=np.uint64)
        offsets[1:] = np.cumsum(padded)[:-1]
        total = int(offsets[-1] + padded[-1]) if n else 0
        self.sizes, self.kinds, self.offsets, self.copy_of = sizes, kinds, offsets, copy_of
        self.total_bytes = int(sizes.sum())
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        arena = torch.empty(total, dtype=torch.uint8, device=device)
        # Fill the whole arena with random bytes, then overwrite float regions
        # with normal values, in chunks so no temporary exceeds ~1 GiB: the
        # normals of consecutive buffers of one dtype are drawn together in
        # float64 (rounded to float32 for float32 buffers) and sliced out.
        chunk = 1 << 30
        for off in range(0, total, chunk):
            m = min(chunk, total - off)
            arena[off:off + m].copy_(torch.randint(0, 256, (m,), dtype=torch.uint8, device=device, generator=gen))
        for kind, dt, es in ((1, torch.float32, 4), (2, torch.float64, 8)):
            idx = [int(i) for i in np.nonzero((kinds == kind) & (copy_of < 0))[0] if int(sizes[i]) >= es]
            start = 0
            while start < len(idx):
                stop, cnt = start, 0
                while stop < len(idx) and (stop == start or cnt + int(sizes[idx[stop]]) // es <= (1 << 27)):
                    cnt += int(sizes[idx[stop]]) // es
                    stop += 1
                vals = torch.randn(cnt, dtype=torch.float64, device=device, generator=gen).to(dt)
                p = 0
                for i in idx[start:stop]:
                    c = int(sizes[i]) // es
                    o = int(offsets[i])
                    arena[o:o + c * es].view(dt).copy_(vals[p:p + c])
                    p += c
                del vals
                start = stop
        for i in np.nonzero(copy_of >= 0)[0]:
            j = int(copy_of[i])
            o, oj, s = int(offsets[i]), int(offsets[j]), int(sizes[i])
            arena[o:o + s].copy_(arena[oj:oj + s])
        self.arena = arena

    def buffer(self, i):
        o, s = int(self.offsets[i]), int(self.sizes[i])
        return self.arena[o:o + s]

    def transfer_log(self, kernel_every=64):
        """The batch as a chronological log: one host-to-device record per
        buffer (host and device addresses from its offset, digest field 0 until
        the digests are written in), and a KERNEL record on device 0 after every
        ``kernel_every`` transfers. Returns (events, index of each buffer's
        record). Copies re-send their source's bytes to the same device, so the
        duplicate count is exactly the number of copies."""
        n = self.sizes.size
        per = kernel_every + 1
        total = n + n // kernel_every
        ev = empty_events(total)
        pos = np.arange(total)
        is_k = (pos % per) == kernel_every
        tx = np.nonzero(~is_k)[0][:n]
        ev["op"] = np.where(is_k, KERNEL, H2D)
        ev["src_dev"], ev["dst_dev"] = HOST, 0
        ev["src_addr"][tx] = np.uint64(HOST_BASE) + self.offsets
        ev["dst_addr"][tx] = np.uint64(DEV_BASE) + self.offsets
        ev["bytes"][tx] = self.sizes
        ev["t_start"] = pos.astype(np.uint64) * np.uint64(1000)
        ev["t_end"] = ev["t_start"] + np.uint64(500)
        return ev, tx

    def pointers(self):
        base = self.arena.data_ptr()
        return (np.uint64(base) + self.offsets).astype(np.uint64)


# ----------------------------------------------------------------------------
# Trace analysis at scale.
# ----------------------------------------------------------------------------
def zipf_finite(rng, s, n_items, size):
    """Draws from a finite Zipf(s) on {0..n_items-1} (rank k has weight 1/(k+1)^s) by inverse CDF."""
    w = 1.0 / np.power(np.arange(1, n_items + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_items - 1)


class TraceAtScale:
    """A chronological log of ``n_map`` map records (ALLOC/H2D/D2H/DELETE) over
    ``n_slots`` variables chosen by a finite Zipf(1.1), plus a KERNEL on device 0
    after every 16 map records (never inside an ALLOC..DELETE pair).

    Units, shuffled: 15% of records re-send the slot's last host-to-device
    digest (planted duplicates), 3% form H2D-D2H-H2D triples of one fresh digest
    (planted round trips), 2% form ALLOC/DELETE pairs of the slot's fixed size at
    its fixed addresses (half with a KERNEL inside, half without: planted unused
    allocations; every pair after a slot's first is a planted repeated
    allocation), the rest are H2D/D2H with fresh, unique 64-bit digests.
    A re-send whose slot has no earlier host-to-device digest becomes a fresh
    H2D. Every interval is disjoint from the others and they increase.

    ``planted`` holds the exact counts the rules must report.
    """

    def __init__(self, seed=4, n_map=10_000_000, n_slots=100_000, zipf_s=1.1, kernel_every=16):
        rng = np.random.default_rng(seed)
        n_rep = int(round(0.15 * n_map))
        n_tri = int(round(0.03 * n_map)) // 3
        n_pair = int(round(0.02 * n_map)) // 2
        n_fresh = n_map - n_rep - 3 * n_tri - 2 * n_pair
        # unit kinds: 0 fresh H2D, 1 fresh D2H, 2 repeat, 3 triple, 4 used pair, 5 unused pair
        fresh_h2d = n_fresh // 2
        kinds = np.concatenate([
            np.zeros(fresh_h2d, np.int8), np.ones(n_fresh - fresh_h2d, np.int8),
            np.full(n_rep, 2, np.int8), np.full(n_tri, 3, np.int8),
            np.full(n_pair // 2, 4, np.int8), np.full(n_pair - n_pair // 2, 5, np.int8)])
        rng.shuffle(kinds)
        n_units = kinds.size
        slots = zipf_finite(rng, zipf_s, n_slots, n_units)
        unit_len = np.array([1, 1, 1, 3, 2, 2], dtype=np.int64)[kinds]  # map records per unit
        # KERNEL after every `kernel_every` map records, placed after the unit that crosses the mark
        map_end = np.cumsum(unit_len)
        map_start = map_end - unit_len
        n_periodic = (map_end // kernel_every) - (map_start // kernel_every)
        inner = (kinds == 4).astype(np.int64)
        rec_len = unit_len + inner + n_periodic
        total = int(rec_len.sum())
        rec_start = np.cumsum(rec_len) - rec_len
        ev = empty_events(total)
        slot_size = np.floor(np.exp(rng.uniform(math.log(8), math.log(1 << 24), size=n_slots))).astype(np.uint64)
        host_addr = np.uint64(HOST_BASE) + np.arange(n_slots, dtype=np.uint64) * np.uint64(1 << 20)
        dev_addr = np.uint64(DEV_BASE) + np.arange(n_slots, dtype=np.uint64) * np.uint64(1 << 20)
        # fresh unique digests: one per fresh unit and one per triple
        n_digests = n_fresh + n_tri
        dg = np.unique(rng.integers(0, 2**63, size=n_digests + 1024, dtype=np.int64).astype(np.uint64)
                       ^ (rng.integers(0, 2, size=n_digests + 1024).astype(np.uint64) << np.uint64(63)))
        while dg.size < n_digests:
            extra = rng.integers(0, 2**63, size=4096, dtype=np.int64).astype(np.uint64)
            dg = np.unique(np.concatenate([dg, extra]))
        dg = dg[:n_digests].copy()
        rng.shuffle(dg)
        has_digest = (kinds <= 1) | (kinds == 3)
        unit_digest = np.zeros(n_units, dtype=np.uint64)
        unit_digest[has_digest] = dg
        # Re-sends: source = last earlier H2D-carrying unit (fresh H2D, triple) in the same slot.
        carries_h2d = (kinds == 0) | (kinds == 3)
        order = np.lexsort((np.arange(n_units), slots))  # by slot, then time
        so_slot = slots[order]
        so_idx = np.where(carries_h2d[order], np.arange(n_units), -1)
        last = np.maximum.accumulate(so_idx)
        # the latest source strictly before each position in slot order
        prev_src = np.empty(n_units, dtype=np.int64)
        prev_src[0] = -1
        prev_src[1:] = last[:-1]
        valid_src = prev_src >= 0
        valid_src[valid_src] &= so_slot[prev_src[valid_src]] == so_slot[valid_src]
        src_unit = np.full(n_units, -1, dtype=np.int64)
        src_unit[order] = np.where(valid_src, order[np.maximum(prev_src, 0)], -1)
        rep = kinds == 2
        orphan = rep & (src_unit < 0)
        # orphans become fresh H2Ds with their own fresh digests
        n_orphan = int(orphan.sum())
        if n_orphan:
            more = rng.integers(0, 2**63, size=n_orphan + 1024, dtype=np.int64).astype(np.uint64) | np.uint64(1 << 63)
            more = np.setdiff1d(np.unique(more), dg)[:n_orphan]
            assert more.size == n_orphan
            perm = rng.permutation(n_orphan)
            unit_digest[orphan] = more[perm]
            kinds = kinds.copy()
            kinds[orphan] = 0
            rep = kinds == 2
        unit_digest[rep] = unit_digest[src_unit[rep]]
        # expand units into records
        u_of_rec = np.repeat(np.arange(n_units), rec_len)
        pos_in_unit = np.arange(total) - rec_start[u_of_rec]
        k = kinds[u_of_rec]
        s = slots[u_of_rec]
        ulen = unit_len[u_of_rec] + inner[u_of_rec]
        is_periodic = pos_in_unit >= ulen
        op = np.zeros(total, dtype=np.uint8)
        op[(k == 0)] = H2D
        op[(k == 1)] = D2H
        op[(k == 2)] = H2D
        tri_pos = np.where(k == 3, pos_in_unit, -1)
        op[tri_pos == 0] = H2D
        op[tri_pos == 1] = D2H
        op[tri_pos == 2] = H2D
        pair_pos = np.where((k == 4) | (k == 5), pos_in_unit, -1)
        op[pair_pos == 0] = ALLOC
        op[(k == 4) & (pair_pos == 1)] = KERNEL
        op[(k == 4) & (pair_pos == 2)] = DELETE
        op[(k == 5) & (pair_pos == 1)] = DELETE
        op[is_periodic] = KERNEL
        ev["op"] = op
        is_tx = (op == H2D) | (op == D2H)
        is_ad = (op == ALLOC) | (op == DELETE)
        is_k = op == KERNEL
        ev["digest"] = np.where(is_tx, unit_digest[u_of_rec], np.uint64(0))
        h2d = op == H2D
        d2h = op == D2H
        ev["src_dev"] = np.where(d2h, 0, HOST).astype(np.int16)
        ev["dst_dev"] = np.where(d2h, HOST, 0).astype(np.int16)
        ha, da = host_addr[s], dev_addr[s]
        ev["src_addr"] = np.where(d2h, da, np.where(is_k, np.uint64(0), ha))
        ev["dst_addr"] = np.where(d2h, ha, np.where(is_k, np.uint64(0), da))
        nbytes = np.where(is_k, np.uint64(0), slot_size[s])
        ev["bytes"] = nbytes
        ev["codeptr"] = np.uint64(0x403000) + (k.astype(np.uint64) << np.uint64(4))
        ev["t_start"], ev["t_end"] = _times(rng, total, nbytes, gap_ns=1000.0, base_ns=5000, rate_bytes_per_ns=25.0)
        self.events = ev
        self.n_map = n_map
        n_rep_final = int(rep.sum())
        pair_slots = slots[(kinds == 4) | (kinds == 5)]
        # What the generator planted, record by record. Every interval is
        # disjoint from the others and they increase with the index, so "a
        # KERNEL record lies between two records" is the same as "a kernel runs
        # between them in time".
        dur = (ev["t_end"] - ev["t_start"]).astype(np.uint64)
        rec_dd = ((k == 2) & (pos_in_unit == 0)) | (tri_pos == 2)
        rec_rx = (tri_pos == 1) | (tri_pos == 2)
        pair_units = np.nonzero((kinds == 4) | (kinds == 5))[0]  # in time order
        first_of_slot = np.zeros(pair_units.size, dtype=bool)
        _, first = np.unique(slots[pair_units], return_index=True)
        first_of_slot[first] = True
        alloc_rec = rec_start[pair_units]
        delete_rec = alloc_rec + np.where(kinds[pair_units] == 4, 2, 1)
        pair_dur = dur[alloc_rec] + dur[delete_rec]
        pair_bytes = nbytes[alloc_rec]
        ra = ~first_of_slot
        ua = kinds[pair_units] == 5
        # A host-to-device copy is never read when no KERNEL record follows it
        # before the next copy of its slot (or at all, when none follows).
        kc = np.cumsum(is_k)
        h_idx = np.nonzero(h2d)[0]
        o = np.lexsort((h_idx, s[h_idx]))
        hi, hs = h_idx[o], s[h_idx][o]
        has_next = np.zeros(hi.size, dtype=bool)
        has_next[:-1] = hs[1:] == hs[:-1]
        nxt = np.where(has_next, np.roll(hi, -1), 0)
        between = np.where(has_next, kc[np.maximum(nxt - 1, 0)] - kc[hi], kc[-1] - kc[hi])
        rec_ut = np.zeros(total, dtype=bool)
        rec_ut[hi[between == 0]] = True
        removable = rec_dd | rec_rx | rec_ut
        self.planted = {
            "n_transfers": int(is_tx.sum()),
            "n_kernels": int(is_k.sum()),
            "n_alloc_pairs": n_pair,
            "dd_events": n_rep_final + n_tri,
            "dd_bytes": int(nbytes[rec_dd].sum()),
            "dd_time_ns": int(dur[rec_dd].sum()),
            "rt_pairs": 2 * n_tri,
            "rt_rx_events": 2 * n_tri,
            "rt_bytes": int(nbytes[rec_rx].sum()),
            "rt_time_ns": int(dur[rec_rx].sum()),
            "ra_events": n_pair - int(np.unique(pair_slots).size),
            "ra_bytes": int(pair_bytes[ra].sum()),
            "ra_time_ns": int(pair_dur[ra].sum()),
            "ua_events": n_pair - n_pair // 2,
            "ua_bytes": int(pair_bytes[ua].sum()),
            "ua_time_ns": int(pair_dur[ua].sum()),
            "ut_events": int(rec_ut.sum()),
            "ut_bytes": int(nbytes[rec_ut].sum()),
            "ut_time_ns": int(dur[rec_ut].sum()),
            "elim_ns": int(dur[removable].sum()) + int(pair_dur[ra | ua].sum()),
            "span_ns": int(ev["t_end"][-1] - ev["t_start"][0]),
            "n_unpaired_alloc": 0,
            "n_unpaired_delete": 0,
        }


# ---------------------------------------------------------------------------
# Serving: Poisson arrivals of mapping-event requests with device payloads.
# ---------------------------------------------------------------------------
class ServingSchedule:
    """``n`` requests arriving at ``rate`` per second (exponential gaps), each a
    mapping record whose transfer moves a 256-byte aligned slice of a seeded
    device arena (log-uniform ``lo``..``hi`` bytes). 20% of transfers re-send
    an earlier slice to the same place (duplicates); 3% of records form
    H2D-D2H-H2D triples of one slice (round trips); 2% are ALLOC/DELETE pairs of
    a slot; a KERNEL follows every 16 records.

    ``events`` (digest fields 0: the server fills them from the payloads),
    ``payload_off`` / ``payload_bytes`` (into ``arena``, -1 / 0 for none),
    ``arrival_ns``.
    """

    def __init__(self, seed=5, n=10_000, rate=10_000.0, lo=4096, hi=64 << 20, arena=None, arena_bytes=16 << 30,
                 n_slots=10_000, device="cpu"):
        import torch
        rng = np.random.default_rng(seed)
        if arena is None:
            gen = torch.Generator(device=device)
            gen.manual_seed(seed)
            arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
            chunk = 1 << 30
            for off in range(0, arena_bytes, chunk):
                m = min(chunk, arena_bytes - off)
                arena[off:off + m].copy_(torch.randint(0, 256, (m,), dtype=torch.uint8, device=device, generator=gen))
        self.arena = arena
        asize = arena.numel()
        hi = min(hi, asize)
        ev = empty_events(n)
        off = np.full(n, -1, dtype=np.int64)
        nb = np.zeros(n, dtype=np.uint64)
        slots = zipf_finite(rng, 1.1, n_slots, n)
        last_h2d = {}
        i = 0
        while i < n:
            u = rng.random()
            s = int(slots[i])
            if i % 17 == 16:
                ev["op"][i] = KERNEL
                ev["dst_dev"][i], ev["src_dev"][i] = 0, HOST
                i += 1
                continue
            if u < 0.02 and i + 1 < n:
                for k, op in enumerate((ALLOC, DELETE)):
                    ev["op"][i + k] = op
                    ev["src_dev"][i + k], ev["dst_dev"][i + k] = HOST, 0
                    ev["src_addr"][i + k] = HOST_BASE + s * (1 << 20)
                    ev["dst_addr"][i + k] = DEV_BASE + s * (1 << 20)
                    ev["bytes"][i + k] = 4096 + (s % 64) * 4096
                i += 2
                continue
            if u < 0.05 and i + 2 < n:
                size = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
                o = int(rng.integers(0, (asize - size) // 256 + 1)) * 256
                for k, (op, sd, dd) in enumerate(((H2D, HOST, 0), (D2H, 0, HOST), (H2D, HOST, 0))):
                    ev["op"][i + k] = op
                    ev["src_dev"][i + k], ev["dst_dev"][i + k] = sd, dd
                    off[i + k], nb[i + k] = o, size
                last_h2d[s] = (o, size)
                i += 3
                continue
            if u < 0.25 and s in last_h2d:
                o, size = last_h2d[s]
                op, sd, dd = H2D, HOST, 0
            else:
                size = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
                o = int(rng.integers(0, (asize - size) // 256 + 1)) * 256
                if rng.random() < 0.5:
                    op, sd, dd = H2D, HOST, 0
                    last_h2d[s] = (o, size)
                else:
                    op, sd, dd = D2H, 0, HOST
            ev["op"][i] = op
            ev["src_dev"][i], ev["dst_dev"][i] = sd, dd
            off[i], nb[i] = o, size
            i += 1
        is_tx = off >= 0
        ev["bytes"][is_tx] = nb[is_tx]
        ev["src_addr"] = np.where(is_tx, np.uint64(HOST_BASE) + slots.astype(np.uint64) * np.uint64(1 << 20), ev["src_addr"])
        ev["dst_addr"] = np.where(is_tx, np.uint64(DEV_BASE) + slots.astype(np.uint64) * np.uint64(1 << 20), ev["dst_addr"])
        gaps = rng.exponential(1e9 / rate, size=n)
        arrival = np.cumsum(gaps).astype(np.uint64)
        arrival -= arrival[0]
        ev["t_start"] = arrival
        ev["t_end"] = arrival + np.uint64(5000) + (ev["bytes"] // np.uint64(25)).astype(np.uint64)
        ev["codeptr"] = np.uint64(0x404000)
        self.events, self.payload_off, self.payload_bytes, self.arrival_ns = ev, off, nb, arrival

    def payload_ptrs(self):
        base = np.uint64(self.arena.data_ptr())
        return np.where(self.payload_off >= 0, base + self.payload_off.astype(np.uint64), np.uint64(0))
