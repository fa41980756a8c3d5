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


def test_struct_layouts_match_header():
    # hdgmg_mesh: int, int, ptr, int, ptr, int; hdgmg_opts; hdgmg_info
    assert ctypes.sizeof(hd.Mesh) == 40
    # 4 ints, 2 doubles, 2 ints, a double, 5 ints, padded to 8
    assert ctypes.sizeof(hd.Opts) == 4 * 4 + 8 * 2 + 4 * 2 + 8 + 4 * 5 + 4
    assert ctypes.sizeof(hd.Info) == 4 + 64 * 4 + 4 + 64 * 8 * 2


def test_default_opts_from_library():
    if not os.path.exists(hd.LIB_PATH):
        pytest.skip("library not built")
    o = hd.default_opts()
    assert (o.m_relax, o.m_smooth, o.cycle, o.vcycle_growth) == (1, 1, 1, 2)
    assert o.rtol == 1e-8 and o.atol == 1e-10 and o.max_it == 500
    assert o.oseen == 0 and o.restart == 50
