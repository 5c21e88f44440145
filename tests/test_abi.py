"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/sm.h declares (no device work)."""
import os
import re

from paper_2511_12235_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "sm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    assert set(declared_symbols()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_status_strings():
    L = _lib.lib()
    for code in range(6):
        assert L.sm_status_str(code)


def test_geometry_struct_layout_matches_header():
    import ctypes as C
    # 4 int32, 6 double, 2 int32, 2 pointers, 2 double, 2 int32, 4 double
    assert C.sizeof(_lib.SmGeometry) == 4 * 4 + 6 * 8 + 2 * 4 + 2 * 8 + 2 * 8 + 2 * 4 + 4 * 8
