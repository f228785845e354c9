"""Host-side checks of the C ABI (no GPU): the built library loads and
exports every function include/nd.h declares; the binding's structs match
the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", "nd.h"), os.path.join(ROOT, "include", "nd_roofline.h")]
LIB = os.path.join(ROOT, "paper_2111_10980_amd", "libnd.so")


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(nd_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("nd_plan_create", "nd_plan_sizes", "nd_run", "nd_round_trace", "nd_plan_destroy",
              "nd_release_cached", "nd_status_str", "nd_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnd.so not built")
def test_status_strings_without_gpu():
    import paper_2111_10980_amd as nd
    assert nd.nd_status_str(0) == "ok"
    assert nd.nd_status_str(2) == "malformed graph"
    assert nd.nd_status_str(3).startswith("r-clique key")


def test_struct_layouts():
    import paper_2111_10980_amd as nd
    assert ctypes.sizeof(nd.nd_csr) == 32
    assert ctypes.sizeof(nd.nd_options) == 16
    # 7 u64 + 2 u32 + 8 floats + 2 floats + 2 u32
    assert ctypes.sizeof(nd.nd_stats) == 7 * 8 + 2 * 4 + 8 * 4 + 2 * 4 + 2 * 4


def test_binding_names_match_header():
    import paper_2111_10980_amd as nd
    for n in declared_functions():
        assert hasattr(nd, n), n
