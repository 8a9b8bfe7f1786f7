"""Python binding of libodp.so (the C ABI in include/odp.h).

Argument marshalling only: every step of the digest and the trace analysis runs
in the library's HIP kernels. torch supplies device memory and streams. The
library must be built first (``python -m paper_2601_12713_amd.build`` or
``__graft_entry__.build()``); loading fails loudly when it is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libodp.so")

ODP_OK, ODP_EINVAL, ODP_ERANGE, ODP_ENOMEM, ODP_EHIP, ODP_ECAPACITY = 0, -1, -2, -3, -4, -5
F_DD, F_RT_TX, F_RT_RX, F_RA, F_UA, F_PAIRED, F_UT, F_INVALID = 1, 2, 4, 8, 16, 32, 64, 128

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
REPORT_BYTES = 8 * len(REPORT_FIELDS) + 16  # + predicted_speedup (double), status, first_bad_event

EXPORTS = [
    "odp_digest_buffers", "odp_digest_buffers_noalloc", "odp_digest_buffers_plain", "odp_analyze_trace",
    "odp_analyze_trace_alg2", "odp_version",
    "odp_last_error_string", "odp_reserve", "odp_release", "odp_device_status",
    "odp_get_tuning", "odp_set_tuning", "odp_server_create", "odp_server_run", "odp_server_drain",
    "odp_server_log", "odp_server_destroy",
]


class OdpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("odp error %d: %s" % (code, msg))
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("split_bytes", ctypes.c_uint32), ("chunk_nodes", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 4)]


_lib = None


def load(path=LIB_PATH):
    """Loads the library (once). Raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libodp.so is not built (%s); run paper_2601_12713_amd/build.py" % path)
    # torch first: the library then binds to the HIP runtime torch already loaded
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    p, sz, u64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
    L.odp_digest_buffers.argtypes = [p, p, sz, p, p]
    L.odp_digest_buffers_noalloc.argtypes = [p, p, sz, p, p]
    L.odp_digest_buffers_plain.argtypes = [p, p, sz, p, p]
    L.odp_analyze_trace.argtypes = [p, sz, p, p, p]
    L.odp_analyze_trace_alg2.argtypes = [p, sz, p, p, p, p, p]
    L.odp_version.argtypes = []
    L.odp_last_error_string.argtypes = []
    L.odp_last_error_string.restype = ctypes.c_char_p
    L.odp_reserve.argtypes = [sz, u64, sz, p]
    L.odp_release.argtypes = []
    L.odp_device_status.argtypes = []
    L.odp_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    L.odp_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    for f in EXPORTS:
        if f != "odp_last_error_string" and not f.startswith("odp_server"):
            getattr(L, f).restype = i32
    _lib = L
    _apply_saved_tuning()
    return L


def _apply_saved_tuning():
    """Applies the autotuner's file for this GPU (tuning/<arch>.json) when present."""
    import torch
    if not torch.cuda.is_available():
        return
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = os.path.join(HERE, "tuning", "%s.json" % arch)
    if os.path.exists(path):
        from . import autotune
        autotune.apply(path)


def _check(code):
    if code != ODP_OK:
        raise OdpError(code, load().odp_last_error_string().decode())
    return code


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def digest_buffers(ptrs, sizes, out, stream=None):
    """Batched digest. ptrs, sizes: int64/uint64 device tensors of n entries; out: int64 device tensor."""
    n = int(sizes.numel())
    _check(load().odp_digest_buffers(_ptr(ptrs), _ptr(sizes), n, _ptr(out), _stream(stream)))
    return out


NOALLOC_MAX_BUFFERS, NOALLOC_MAX_NODES = 16384, 65536


def digest_buffers_noalloc(ptrs, sizes, out, stream=None):
    """Batched digest in the library's fixed device array (no allocation);
    same arguments as digest_buffers."""
    n = int(sizes.numel())
    _check(load().odp_digest_buffers_noalloc(_ptr(ptrs), _ptr(sizes), n, _ptr(out), _stream(stream)))
    return out


def digest_buffers_plain(host_ptrs, host_sizes, out, stream=None):
    """Per-buffer launches. host_ptrs, host_sizes: sequences of ints (device addresses, bytes)."""
    n = len(host_sizes)
    hp = np.ascontiguousarray(np.asarray(host_ptrs, dtype=np.uint64))
    hs = np.ascontiguousarray(np.asarray(host_sizes, dtype=np.uint64))
    _check(load().odp_digest_buffers_plain(ctypes.c_void_p(hp.ctypes.data), ctypes.c_void_p(hs.ctypes.data), n,
                                           _ptr(out), _stream(stream)))
    return out


def digest_tensors(tensors, stream=None, plain=False):
    """Convenience: D64 of each tensor's bytes. Returns a uint64 numpy array (synchronises)."""
    import torch
    dev = tensors[0].device if tensors else torch.device("cuda")
    n = len(tensors)
    ptrs = [t.data_ptr() for t in tensors]
    sizes = [t.numel() * t.element_size() for t in tensors]
    out = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    if plain:
        digest_buffers_plain(ptrs, sizes, out, stream)
    else:
        dp = torch.tensor(np.array(ptrs, dtype=np.uint64).view(np.int64), device=dev)
        ds = torch.tensor(np.array(sizes, dtype=np.uint64).view(np.int64), device=dev)
        digest_buffers(dp, ds, out, stream)
    torch.cuda.synchronize(dev)
    return out[:n].cpu().numpy().view(np.uint64)


def analyze_trace(events, out_flags, out_report, stream=None, n=None):
    """events: device tensor holding n 64-byte records; out_flags: uint8 device tensor (n);
    out_report: device tensor of at least REPORT_BYTES bytes."""
    if n is None:
        n = events.numel() * events.element_size() // 64
    _check(load().odp_analyze_trace(_ptr(events), n, _ptr(out_flags), _ptr(out_report), _stream(stream)))


def analyze_trace_alg2(events, out_flags, out_report, out_rx, out_npairs, stream=None, n=None):
    """analyze_trace plus the pairs the literal Algorithm 2 records: out_rx (int32/uint32 device
    tensor, n) gets the rx record of each recorded tx, else 0xFFFFFFFF; out_npairs (one 64-bit
    device word) their number."""
    if n is None:
        n = events.numel() * events.element_size() // 64
    _check(load().odp_analyze_trace_alg2(_ptr(events), n, _ptr(out_flags), _ptr(out_report), _ptr(out_rx),
                                         _ptr(out_npairs), _stream(stream)))


def report_to_dict(buf):
    """Decodes an odp_report from host bytes (numpy uint8 array or bytes)."""
    raw = np.frombuffer(bytes(buf)[:REPORT_BYTES], dtype=np.uint8)
    vals = raw[:8 * len(REPORT_FIELDS)].view(np.uint64)
    d = {f: int(v) for f, v in zip(REPORT_FIELDS, vals)}
    tail = raw[8 * len(REPORT_FIELDS):]
    d["predicted_speedup"] = float(tail[:8].view(np.float64)[0])
    d["status"] = int(tail[8:12].view(np.int32)[0])
    d["first_bad_event"] = int(tail[12:16].view(np.uint32)[0])
    return d


def reserve(max_buffers=0, max_total_bytes=0, max_events=0, stream=None):
    _check(load().odp_reserve(max_buffers, max_total_bytes, max_events, _stream(stream)))


def release():
    _check(load().odp_release())


def device_status():
    return int(load().odp_device_status())


def get_tuning():
    t = Tuning()
    _check(load().odp_get_tuning(ctypes.byref(t)))
    return {"blocks_per_cu": int(t.blocks_per_cu), "use_graph": int(t.use_graph), "split_bytes": int(t.split_bytes),
            "chunk_nodes": int(t.chunk_nodes)}


def set_tuning(blocks_per_cu=None, use_graph=None, split_bytes=None, chunk_nodes=None):
    t = Tuning()
    _check(load().odp_get_tuning(ctypes.byref(t)))
    if blocks_per_cu is not None:
        t.blocks_per_cu = blocks_per_cu
    if use_graph is not None:
        t.use_graph = int(use_graph)
    if split_bytes is not None:
        t.split_bytes = int(split_bytes)
    if chunk_nodes is not None:
        t.chunk_nodes = int(chunk_nodes)
    _check(load().odp_set_tuning(ctypes.byref(t)))


def version():
    return int(load().odp_version())


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
class _ServerConfig(ctypes.Structure):
    _fields_ = [("max_events", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("max_tick", ctypes.c_uint32),
                ("mode", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


SERVER_BATCHED, SERVER_PLAIN = 0, 1


class _ServerStats(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("ticks", ctypes.c_uint64), ("max_tick", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("budget_waits", ctypes.c_uint64), ("state_bytes", ctypes.c_uint64)]


def _load_server():
    L = load()
    if not getattr(L, "_server_ready", False):
        p, sz = ctypes.c_void_p, ctypes.c_size_t
        L.odp_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
        L.odp_server_run.argtypes = [p, p, p, p, p, sz, p, ctypes.POINTER(_ServerStats)]
        L.odp_server_drain.argtypes = [p, p, p, p]
        L.odp_server_log.argtypes = [p, p, ctypes.POINTER(ctypes.c_size_t)]
        L.odp_server_destroy.argtypes = [p]
        for f in ("odp_server_create", "odp_server_run", "odp_server_drain", "odp_server_log", "odp_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L._server_ready = True
    return L


class Server:
    """Request server (odp_server_*): open-loop schedules, drain, log."""

    def __init__(self, max_events, budget_bytes, max_inflight=1 << 20, max_tick=1024, mode=SERVER_BATCHED):
        L = _load_server()
        cfg = _ServerConfig(max_events, budget_bytes, max_inflight, max_tick, mode, 0)
        h = ctypes.c_void_p()
        _check(L.odp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._n = 0

    def run(self, events, payload_ptrs, payload_bytes, arrival_ns):
        """Returns (complete_ns uint64 array, stats dict). Blocks until done."""
        L = _load_server()
        ev = np.ascontiguousarray(events)
        n = ev.shape[0]
        pp = np.ascontiguousarray(payload_ptrs, dtype=np.uint64)
        pb = np.ascontiguousarray(payload_bytes, dtype=np.uint64)
        an = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        done = np.zeros(max(n, 1), dtype=np.uint64)
        st = _ServerStats()
        _check(L.odp_server_run(self._h, ctypes.c_void_p(ev.ctypes.data), ctypes.c_void_p(pp.ctypes.data),
                                ctypes.c_void_p(pb.ctypes.data), ctypes.c_void_p(an.ctypes.data), n,
                                ctypes.c_void_p(done.ctypes.data), ctypes.byref(st)))
        self._n += n
        return done[:n], {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def drain(self):
        """Returns (flags decided before the drain, final flags, final report dict) as host arrays."""
        import torch
        L = _load_server()
        n = self._n
        imm = torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
        fl = torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
        rep = torch.zeros(REPORT_BYTES, dtype=torch.uint8, device="cuda")
        _check(L.odp_server_drain(self._h, _ptr(imm), _ptr(fl), _ptr(rep)))
        return imm[:n].cpu().numpy(), fl[:n].cpu().numpy(), report_to_dict(rep.cpu().numpy())

    def log(self):
        """The logged records (digests filled in) as a uint8 host array of n*64 bytes."""
        import torch
        L = _load_server()
        cnt = ctypes.c_size_t()
        _check(L.odp_server_log(self._h, None, ctypes.byref(cnt)))
        buf = torch.zeros(max(cnt.value, 1) * 64, dtype=torch.uint8, device="cuda")
        _check(L.odp_server_log(self._h, _ptr(buf), ctypes.byref(cnt)))
        return buf[:cnt.value * 64].cpu().numpy()

    def close(self):
        if self._h:
            _load_server().odp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
