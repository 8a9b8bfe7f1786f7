"""Serial CPU oracle (ctypes binding to oracle/odp_oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.

Parity status of each function (how it is pinned, see tests/test_oracle_*.py):
  xxh64        pinned: the independent python ``xxhash`` package on random
               inputs of every length class (0..4096+ bytes, several seeds).
  d64          pinned: an independent composition of ``xxhash`` calls written
               in the test, over one-, two- and three-level trees; invariants.
  analyze      pinned: O(n^2) brute force over Defs. 1-4 using byte equality of
               real payloads on random tiny traces (every flag and every count
               and sum of the report, unused transfers and the
               optimization-potential figures included); hand traces of the
               paper's Listings 1 and 2 and of each unused-transfer case;
               closed forms for alternating round-trip chains and repeated
               copies; planted counts and sums of the synthetic generators.
  alg2_pairs   the pairs Algorithm 2 records; pinned by hand traces and by
               its agreement with the round-trip rule on two endpoints.
  The counts in the paper's issue table are not reproducible here (the
  applications are absent): parity unpinned for those.
"""
import ctypes
import os

import numpy as np

from . import build as _build

F_DD, F_RT_TX, F_RT_RX, F_RA, F_UA, F_PAIRED, F_UT, F_INVALID = 1, 2, 4, 8, 16, 32, 64, 128
OP_ALLOC, OP_H2D, OP_D2H, OP_D2D, OP_DELETE, OP_KERNEL = 1, 2, 3, 4, 5, 6

REPORT_FIELDS = [
    "n_events", "n_invalid", "n_transfers", "n_kernels",
    "n_alloc_pairs", "n_unpaired_alloc", "n_unpaired_delete",
    "dd_events", "dd_groups", "dd_members", "dd_bytes", "dd_time_ns",
    "rt_pairs", "rt_rx_events", "rt_bytes", "rt_time_ns",
    "ra_events", "ra_groups", "ra_members", "ra_bytes", "ra_time_ns",
    "ua_events", "ua_bytes", "ua_time_ns",
    "ut_events", "ut_bytes", "ut_time_ns",
    "span_ns", "elim_ns",
]


class _Report(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in REPORT_FIELDS] + [
        ("predicted_speedup", ctypes.c_double), ("status", ctypes.c_int32), ("first_bad_event", ctypes.c_uint32)]


_lib = None


def use_native_build(directory):
    """Loads a copy compiled with -march=native for this host (built into
    `directory`) in place of the portable build; used to time the oracle as a
    CPU baseline. Same source, same results."""
    global _lib
    _lib = None
    return lib(_build.build_native(directory))


def lib(path=None):
    global _lib
    if _lib is None:
        path = path or _build.build(force=False)
        L = ctypes.CDLL(path)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        L.orc_xxh64.restype = u64
        L.orc_xxh64.argtypes = [p, u64, u64]
        L.orc_d64.restype = u64
        L.orc_d64.argtypes = [p, u64]
        L.orc_d64_many.restype = None
        L.orc_d64_many.argtypes = [p, p, u64, p]
        L.orc_analyze.restype = ctypes.c_int
        L.orc_analyze.argtypes = [p, u64, p, ctypes.POINTER(_Report)]
        L.orc_alg2_pairs.restype = ctypes.c_int64
        L.orc_alg2_pairs.argtypes = [p, p, u64, p, p]
        _lib = L
    return _lib


def _bytes_view(data):
    a = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray, memoryview)) else data)
    return a.view(np.uint8).reshape(-1), a


def xxh64(data, seed=0):
    """XXH64 of a byte string (public xxHash specification)."""
    b, keep = _bytes_view(data)
    return int(lib().orc_xxh64(b.ctypes.data, b.size, seed))


def d64(data):
    """ODP-D64 v1 digest of a byte string."""
    b, keep = _bytes_view(data)
    return int(lib().orc_d64(b.ctypes.data, b.size))


def d64_many(buffers):
    """ODP-D64 v1 of each buffer in a list of byte arrays; returns uint64 array."""
    views = [_bytes_view(x)[0] for x in buffers]
    n = len(views)
    ptrs = (ctypes.c_void_p * max(n, 1))(*[v.ctypes.data for v in views])
    sizes = np.array([v.size for v in views], dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_d64_many(ctypes.cast(ptrs, ctypes.c_void_p), sizes.ctypes.data, n, out.ctypes.data)
    return out


def _events(events):
    a = np.ascontiguousarray(events)
    if a.dtype.itemsize != 64:
        raise ValueError("event records are 64 bytes each")
    return a


def analyze(events):
    """Run the detection rules over a chronological event log.

    ``events`` is any contiguous numpy array of 64-byte event records.
    Returns (flags uint8[n], report dict).
    """
    a = _events(events)
    n = a.shape[0]
    flags = np.zeros(n, dtype=np.uint8)
    rep = _Report()
    lib().orc_analyze(a.ctypes.data, n, flags.ctypes.data, ctypes.byref(rep))
    d = {f: int(getattr(rep, f)) for f in REPORT_FIELDS}
    d["predicted_speedup"] = float(rep.predicted_speedup)
    d["status"] = int(rep.status)
    d["first_bad_event"] = int(rep.first_bad_event)
    return flags, d


def alg2_pairs(events, idx):
    """The pairs Algorithm 2 records over the transfers ``idx``: list of (tx_position, rx_position)."""
    a = _events(events)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    tx = np.zeros(max(idx.size, 1), dtype=np.int64)
    rx = np.zeros(max(idx.size, 1), dtype=np.int64)
    npairs = lib().orc_alg2_pairs(a.ctypes.data, idx.ctypes.data, idx.size, tx.ctypes.data, rx.ctypes.data)
    return list(zip(tx[:npairs].tolist(), rx[:npairs].tolist()))


def unused_transfers(events):
    """Unused transfers (Def. 4, transfer half): uint8 per record, 1 when flagged."""
    flags, _ = analyze(events)
    return ((flags & F_UT) != 0).astype(np.uint8)
