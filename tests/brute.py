"""O(n^2) brute force over the paper's definitions (Sec. 4, Defs. 1-4), with
equality of transferred data decided by comparing the BYTES moved, not digests
(the paper's collision-check idea, App. B), and the optimization-potential
figures of Sec. 7.6 summed from the flags it finds. Used only on tiny traces.

Every count and sum of the report is recomputed here from the definitions:
  * duplicates, round trips, pairs, repeated and unused allocations as in
    Defs. 1-4, with bytes and durations summed over the flagged records (a
    repeated or unused allocation adds its DELETE's duration: the allocation's
    whole lifetime is the mapping the pattern concerns);
  * unused transfers by quantifying over kernels: a copy into device memory is
    used when some kernel on that device is still running or not yet started
    when the copy begins, and starts no later than the next copy to the same
    place (in log order) begins to overwrite it (closed intervals: touching
    counts as use).
"""
ALLOC, H2D, D2H, D2D, DELETE, KERNEL = 1, 2, 3, 4, 5, 6
F_DD, F_RT_TX, F_RT_RX, F_RA, F_UA, F_PAIRED, F_UT, F_INVALID = 1, 2, 4, 8, 16, 32, 64, 128


def _valid(ev, i):
    e = ev[i]
    op = int(e["op"])
    if op < 1 or op > 6:
        return False
    if int(e["t_end"]) < int(e["t_start"]):
        return False
    if i > 0 and int(e["t_start"]) < int(ev[i - 1]["t_start"]):
        return False
    if not (-1 <= int(e["dst_dev"]) <= 9):
        return False
    if op in (H2D, D2H, D2D) and not (-1 <= int(e["src_dev"]) <= 9):
        return False
    return True


def brute(ev, data_of):
    """``data_of(i)`` returns the bytes transfer i moved. Returns (flags list, counts dict)."""
    n = len(ev)
    valid = [_valid(ev, i) for i in range(n)]
    flags = [0 if valid[i] else F_INVALID for i in range(n)]
    op = [int(ev[i]["op"]) for i in range(n)]
    src = [int(ev[i]["src_dev"]) for i in range(n)]
    dst = [int(ev[i]["dst_dev"]) for i in range(n)]
    ts = [int(ev[i]["t_start"]) for i in range(n)]
    te = [int(ev[i]["t_end"]) for i in range(n)]
    nbytes = [int(ev[i]["bytes"]) for i in range(n)]
    dur = [te[i] - ts[i] for i in range(n)]
    T = [i for i in range(n) if valid[i] and op[i] in (H2D, D2H, D2D)]
    K = [i for i in range(n) if valid[i] and op[i] == KERNEL]
    data = {i: bytes(data_of(i)) for i in T}
    c = dict(dd_events=0, dd_groups=0, dd_members=0, dd_bytes=0, dd_time_ns=0,
             rt_pairs=0, rt_rx_events=0, rt_bytes=0, rt_time_ns=0,
             n_alloc_pairs=0, ra_events=0, ra_groups=0, ra_members=0, ra_bytes=0, ra_time_ns=0,
             ua_events=0, ua_bytes=0, ua_time_ns=0, ut_events=0, ut_bytes=0, ut_time_ns=0,
             n_unpaired_alloc=0, n_unpaired_delete=0, n_transfers=len(T), n_kernels=len(K),
             n_invalid=sum(1 for v in valid if not v))
    # Def. 1: a receiver gets data it already received.
    for i in T:
        if any(j < i and dst[j] == dst[i] and data[j] == data[i] for j in T):
            flags[i] |= F_DD
            c["dd_events"] += 1
            c["dd_bytes"] += nbytes[i]
            c["dd_time_ns"] += dur[i]
    groups = {}
    for i in T:
        key = None
        for g in groups:
            if dst[g] == dst[i] and data[g] == data[i]:
                key = g
                break
        groups.setdefault(i if key is None else key, []).append(i)
    for g, mem in groups.items():
        if len(mem) >= 2:
            c["dd_groups"] += 1
            c["dd_members"] += len(mem)
    # Def. 2: A sends to B, and later A receives the same data back from B.
    NS = [i for i in T if src[i] != dst[i]]
    for i in NS:
        later = [j for j in NS if j > i and data[j] == data[i] and src[j] == dst[i] and dst[j] == src[i]]
        if later:
            flags[i] |= F_RT_TX
            c["rt_pairs"] += 1
            flags[later[0]] |= F_RT_RX  # the return leg completing the earliest trip
    for i in NS:
        if flags[i] & F_RT_RX:
            c["rt_rx_events"] += 1
            c["rt_bytes"] += nbytes[i]
            c["rt_time_ns"] += dur[i]
    # Pairing: a DELETE and the latest earlier ALLOC/DELETE at the same (device, device address), if an ALLOC.
    AD = [i for i in range(n) if valid[i] and op[i] in (ALLOC, DELETE)]
    pairs = []
    for d in AD:
        if op[d] != DELETE:
            continue
        prev = [j for j in AD if j < d and dst[j] == dst[d] and int(ev[j]["dst_addr"]) == int(ev[d]["dst_addr"])]
        if prev and op[prev[-1]] == ALLOC:
            pairs.append((prev[-1], d))
            flags[prev[-1]] |= F_PAIRED
            flags[d] |= F_PAIRED
    pairs.sort()
    c["n_alloc_pairs"] = len(pairs)
    c["n_unpaired_alloc"] = sum(1 for i in AD if op[i] == ALLOC and not flags[i] & F_PAIRED)
    c["n_unpaired_delete"] = sum(1 for i in AD if op[i] == DELETE and not flags[i] & F_PAIRED)

    def rkey(a):
        return (int(ev[a]["src_addr"]), dst[a], nbytes[a])

    # Def. 3: the same variable allocated (and deleted) more than once.
    for a, d in pairs:
        if any(b < a and rkey(b) == rkey(a) for b, _ in pairs):
            flags[a] |= F_RA
            c["ra_events"] += 1
            c["ra_bytes"] += nbytes[a]
            c["ra_time_ns"] += dur[a] + dur[d]
    keys = {}
    for a, _ in pairs:
        keys.setdefault(rkey(a), []).append(a)
    for k, mem in keys.items():
        if len(mem) >= 2:
            c["ra_groups"] += 1
            c["ra_members"] += len(mem)
    # Def. 4 (allocation half): the lifetime meets no kernel execution on that device.
    for a, d in pairs:
        A, D = ts[a], te[d]
        used = any(dst[k] == dst[a] and ts[k] <= D and te[k] >= A for k in K)
        if not used:
            flags[a] |= F_UA
            c["ua_events"] += 1
            c["ua_bytes"] += nbytes[a]
            c["ua_time_ns"] += dur[a] + dur[d]
    # Def. 4 (transfer half): a copy into device memory that no kernel on the
    # device can read before a later copy to the same place starts, or ever.
    into = [i for i in T if op[i] in (H2D, D2D) and dst[i] >= 0]

    def place(i):
        return (dst[i], src[i], int(ev[i]["src_addr"]))

    for i in into:
        overwrites = [j for j in into if j > i and place(j) == place(i)]  # later copies, log order
        nxt = overwrites[0] if overwrites else None
        read = any(dst[k] == dst[i] and te[k] >= ts[i] and (nxt is None or ts[k] <= ts[nxt]) for k in K)
        if not read:
            flags[i] |= F_UT
            c["ut_events"] += 1
            c["ut_bytes"] += nbytes[i]
            c["ut_time_ns"] += dur[i]
    # Sec. 7.6: removable time (each record once), span of the log, predicted speedup.
    elim = sum(dur[i] for i in T if flags[i] & (F_DD | F_RT_RX | F_UT))
    elim += sum(dur[a] + dur[d] for a, d in pairs if flags[a] & (F_RA | F_UA))
    V = [i for i in range(n) if valid[i]]
    span = (max(te[i] for i in V) - min(ts[i] for i in V)) if V else 0
    c["span_ns"] = span
    c["elim_ns"] = elim
    c["predicted_speedup"] = 1.0 if span == 0 else (float("inf") if elim >= span else span / (span - elim))
    return flags, c
