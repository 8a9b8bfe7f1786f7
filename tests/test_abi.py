"""CPU checks of the C ABI library: it loads and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "odp.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(odp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_contract():
    names = declared_functions()
    for f in ["odp_digest_buffers", "odp_analyze_trace", "odp_digest_buffers_plain", "odp_reserve",
              "odp_release", "odp_version", "odp_last_error_string"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2601_12713_amd import odp
    if not os.path.exists(odp.LIB_PATH):
        pytest.skip("libodp.so not built")
    lib = ctypes.CDLL(odp.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f), f
    assert set(odp.EXPORTS) == set(declared_functions())


def test_event_record_layout_matches_header():
    from paper_2601_12713_amd import workloads as W
    dt = W.EVENT_DTYPE
    assert dt.itemsize == 64
    assert [dt.fields[f][1] for f in ["digest", "src_addr", "dst_addr", "bytes", "t_start", "t_end", "codeptr",
                                      "src_dev", "dst_dev", "op"]] == [0, 8, 16, 24, 32, 40, 48, 56, 58, 60]


def _lib():
    from paper_2601_12713_amd import odp
    if not os.path.exists(odp.LIB_PATH):
        pytest.skip("libodp.so not built")
    L = ctypes.CDLL(odp.LIB_PATH)
    L.odp_last_error_string.restype = ctypes.c_char_p
    return L


# Argument checks that the entry points make on the host before any device
# call: they run without a GPU.
def test_range_errors_before_any_device_call():
    L = _lib()
    big = ctypes.c_size_t(1 << 32)
    fake = ctypes.c_void_p(0x1000)
    L.odp_reserve.argtypes = [ctypes.c_size_t, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p]
    assert L.odp_reserve(big, 0, 0, None) == -2
    assert L.odp_reserve(0, 0, big, None) == -2
    assert b"2^32" in L.odp_last_error_string()
    L.odp_analyze_trace.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert L.odp_analyze_trace(fake, big, fake, fake, None) == -2
    L.odp_analyze_trace_alg2.argtypes = [ctypes.c_void_p, ctypes.c_size_t] + [ctypes.c_void_p] * 5
    assert L.odp_analyze_trace_alg2(fake, big, fake, fake, fake, fake, None) == -2
    for f in (L.odp_digest_buffers, L.odp_digest_buffers_plain):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
        assert f(fake, fake, big, fake, None) == -2
    L.odp_digest_buffers_noalloc.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_size_t] + [ctypes.c_void_p] * 2
    assert L.odp_digest_buffers_noalloc(fake, fake, 16385, fake, None) == -2
    assert b"maximum" in L.odp_last_error_string()


def test_invalid_arguments_before_any_device_call():
    L = _lib()
    fake = ctypes.c_void_p(0x1000)
    L.odp_analyze_trace.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert L.odp_analyze_trace(None, 5, fake, fake, None) == -1      # null events with n > 0
    assert L.odp_analyze_trace(fake, 5, fake, None, None) == -1      # null report
    L.odp_analyze_trace_alg2.argtypes = [ctypes.c_void_p, ctypes.c_size_t] + [ctypes.c_void_p] * 5
    assert L.odp_analyze_trace_alg2(fake, 5, fake, fake, fake, None, None) == -1   # null pair count
    assert L.odp_analyze_trace_alg2(fake, 5, fake, fake, None, fake, None) == -1   # null rx with n > 0
    for f in (L.odp_digest_buffers, L.odp_digest_buffers_noalloc, L.odp_digest_buffers_plain):
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
        assert f(None, fake, 3, fake, None) == -1
        assert f(fake, fake, 0, None, None) == 0                      # n = 0: nothing to do
    L.odp_set_tuning.argtypes = [ctypes.c_void_p]
    bad = (ctypes.c_uint32 * 8)(9, 1, 0, 0, 0, 0, 0, 0)              # 9 workgroups per CU
    assert L.odp_set_tuning(bad) == -1
    bad = (ctypes.c_uint32 * 8)(4, 1, 100, 0, 0, 0, 0, 0)            # split below one leaf
    assert L.odp_set_tuning(bad) == -1
    bad = (ctypes.c_uint32 * 8)(4, 1, 0, 17, 0, 0, 0, 0)             # 17 items per claim
    assert L.odp_set_tuning(bad) == -1
    L.odp_server_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    h = ctypes.c_void_p()
    cfg = (ctypes.c_uint64 * 2)(0, 1 << 20)
    raw = bytes(cfg) + bytes((ctypes.c_uint32 * 4)(8, 16, 0, 0))   # max_events 0
    assert L.odp_server_create(ctypes.c_char_p(raw), ctypes.byref(h)) == -2
    raw = bytes((ctypes.c_uint64 * 2)(8, 1 << 20)) + bytes((ctypes.c_uint32 * 4)(8, 2000, 0, 0))  # max_tick
    assert L.odp_server_create(ctypes.c_char_p(raw), ctypes.byref(h)) == -1
