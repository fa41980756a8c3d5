"""CPU checks of the HIP library: it loads and exports every symbol that
include/hdgmg.h declares, and its ctypes structures match the header."""
import ctypes
import os
import re

import pytest

import paper_2303_06762_amd as hd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hdgmg.h")).read()
    pat = r"^(?:hdgmg_status|void|const char\*)\s+(hdgmg_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(pat, src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(hd.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(hd.LIB_PATH)
    names = declared_symbols()
    assert set(names) == set(hd.SYMBOLS)
    for n in names:
        assert hasattr(L, n), n


def _c_layouts(tmp_path):
    """sizeof and field offsets of the header's structs, from a C program
    compiled against include/hdgmg.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields = {"hdgmg_mesh": [f for f, _ in hd.Mesh._fields_],
              "hdgmg_opts": [f for f, _ in hd.Opts._fields_],
              "hdgmg_info": [f for f, _ in hd.Info._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hdgmg.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.strip().splitlines()}


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of hdgmg_mesh, hdgmg_opts and hdgmg_info against the
    # C compiler's layout of the header (sizes and every field offset)
    c = _c_layouts(tmp_path)
    for name, cls in (("hdgmg_mesh", hd.Mesh), ("hdgmg_opts", hd.Opts), ("hdgmg_info", hd.Info)):
        assert c[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert c[(name, f)] == getattr(cls, f).offset, (name, f)


def test_allocator_callbacks_are_c_compatible():
    # null callbacks (the library's own hipMalloc) and the torch allocator's
    # callbacks convert to the setup's argument types
    assert not hd.ALLOC_FN() and not hd.FREE_FN()
    assert ctypes.cast(hd.ALLOC_FN(lambda n, c: None), ctypes.c_void_p).value


def test_default_opts_from_library():
    if not os.path.exists(hd.LIB_PATH):
        pytest.skip("library not built")
    o = hd.default_opts()
    assert (o.m_relax, o.m_smooth, o.cycle, o.vcycle_growth) == (1, 1, 1, 2)
    assert o.rtol == 1e-8 and o.atol == 1e-10 and o.max_it == 500
    assert o.oseen == 0 and o.restart == 50
