"""Parser for the hand-written worked-example traces under tests/golden/."""
import os

import numpy as np

from paper_2601_12713_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
OPS = {"ALLOC": W.ALLOC, "H2D": W.H2D, "D2H": W.D2H, "D2D": W.D2D, "DELETE": W.DELETE, "KERNEL": W.KERNEL}


def load(name):
    """Returns (events, payload list, payload_of, expected counts)."""
    contents, recs, expect = {}, [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "content":
                assert tok[2] == "int32"
                contents[tok[1]] = np.array([int(x) for x in tok[3:]], dtype="<i4").tobytes()
            elif tok[0] == "expect":
                for kv in tok[1:]:
                    k, v = kv.split("=")
                    expect[k] = int(v)
            else:
                recs.append((OPS[tok[0]], tok[1], tok[2]))
    names = sorted({v for _, v, _ in recs if v != "-"})
    var_id = {v: i for i, v in enumerate(names)}
    payload_names = list(contents)
    payloads = [contents[p] for p in payload_names]
    n = len(recs)
    ev = W.empty_events(n)
    payload_of = np.full(n, -1, dtype=np.int64)
    for i, (op, var, content) in enumerate(recs):
        ev["op"][i] = op
        ev["t_start"][i] = 100 * i
        ev["t_end"][i] = 100 * i + 50
        ev["codeptr"][i] = 0x1000 + i
        if op == W.KERNEL:
            ev["src_dev"][i], ev["dst_dev"][i] = -1, 0
            continue
        v = var_id[var]
        ha, da = W.HOST_BASE + v * 4096, W.DEV_BASE + v * 4096
        if op == W.D2H:
            ev["src_dev"][i], ev["dst_dev"][i] = 0, -1
            ev["src_addr"][i], ev["dst_addr"][i] = da, ha
        else:
            ev["src_dev"][i], ev["dst_dev"][i] = -1, 0
            ev["src_addr"][i], ev["dst_addr"][i] = ha, da
        if content != "-":
            payload_of[i] = payload_names.index(content)
            ev["bytes"][i] = len(payloads[payload_of[i]])
        else:
            ev["bytes"][i] = 16 if var == "a" else (20 if var == "a" else 4)
    # allocations of `a` carry a's size so that the RA key (host addr, device, bytes) is stable
    for i, (op, var, _) in enumerate(recs):
        if op in (W.ALLOC, W.DELETE):
            sz = [len(payloads[payload_of[j]]) for j in range(n) if recs[j][1] == var and payload_of[j] >= 0]
            ev["bytes"][i] = sz[0] if sz else 4
    return ev, payloads, payload_of, expect
