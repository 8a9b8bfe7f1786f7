"""O(n^2) brute force over the paper's definitions (Sec. 4, Defs. 1-4), with
equality of transferred data decided by comparing the BYTES moved, not digests
(the paper's collision-check idea, App. B). Used only on tiny traces.
"""
ALLOC, H2D, D2H, D2D, DELETE, KERNEL = 1, 2, 3, 4, 5, 6
F_DD, F_RT_TX, F_RT_RX, F_RA, F_UA, F_PAIRED, F_INVALID = 1, 2, 4, 8, 16, 32, 128


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
    T = [i for i in range(n) if valid[i] and op[i] in (H2D, D2H, D2D)]
    data = {i: bytes(data_of(i)) for i in T}
    c = dict(dd_events=0, dd_groups=0, dd_members=0, rt_pairs=0, rt_rx_events=0,
             n_alloc_pairs=0, ra_events=0, ra_groups=0, ra_members=0, ua_events=0,
             n_unpaired_alloc=0, n_unpaired_delete=0, n_transfers=len(T),
             n_kernels=sum(1 for i in range(n) if valid[i] and op[i] == KERNEL),
             n_invalid=sum(1 for v in valid if not v))
    # Def. 1: a receiver gets data it already received.
    for i in T:
        if any(j < i and dst[j] == dst[i] and data[j] == data[i] for j in T):
            flags[i] |= F_DD
            c["dd_events"] += 1
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
    c["rt_rx_events"] = sum(1 for i in NS if flags[i] & F_RT_RX)
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
        return (int(ev[a]["src_addr"]), dst[a], int(ev[a]["bytes"]))

    # Def. 3: the same variable allocated (and deleted) more than once.
    for a, _ in pairs:
        if any(b < a and rkey(b) == rkey(a) for b, _ in pairs):
            flags[a] |= F_RA
            c["ra_events"] += 1
    keys = {}
    for a, _ in pairs:
        keys.setdefault(rkey(a), []).append(a)
    for k, mem in keys.items():
        if len(mem) >= 2:
            c["ra_groups"] += 1
            c["ra_members"] += len(mem)
    # Def. 4 (allocation half): the lifetime meets no kernel execution on that device.
    K = [i for i in range(n) if valid[i] and op[i] == KERNEL]
    for a, d in pairs:
        A, D = int(ev[a]["t_start"]), int(ev[d]["t_end"])
        used = any(dst[k] == dst[a] and int(ev[k]["t_start"]) <= D and int(ev[k]["t_end"]) >= A for k in K)
        if not used:
            flags[a] |= F_UA
            c["ua_events"] += 1
    return flags, c
