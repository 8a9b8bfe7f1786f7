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
