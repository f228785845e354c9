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
    # 6 x 32-bit + 2 u64 + 4 x 32-bit
    assert ctypes.sizeof(nd.nd_options) == 6 * 4 + 2 * 8 + 4 * 4
    # 7 u64 + 2 u32 + 8 floats + 2 floats + 2 u32 + 4 u64 + 2 u32
    assert ctypes.sizeof(nd.nd_stats) == 7 * 8 + 2 * 4 + 8 * 4 + 2 * 4 + 2 * 4 + 4 * 8 + 2 * 4


def test_struct_layouts_match_c(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a
    C compiler makes of include/nd.h."""
    import shutil
    import subprocess
    import paper_2111_10980_amd as nd
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"nd_csr": nd.nd_csr, "nd_options": nd.nd_options, "nd_stats": nd.nd_stats,
               "nd_roofline": nd.nd_roofline, "nd_tune_report": nd.nd_tune_report}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "nd.h"',
             '#include "nd_roofline.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'  printf("{sname} %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{sname}.{fname} %zu\\n", offsetof({sname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for sname, cls in structs.items():
        assert int(got[sname]) == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(got[f"{sname}.{fname}"]) == getattr(cls, fname).offset, (sname, fname)


def test_binding_names_match_header():
    import paper_2111_10980_amd as nd
    for n in declared_functions():
        assert hasattr(nd, n), n
