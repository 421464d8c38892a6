"""CPU checks of the C ABI: the library loads and exports every declared symbol, and
argument errors are reported without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1011_4046_amd import semipar as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semipar.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("region_init_from_surfaces", "region_evolve", "region_emit_final_surfaces",
              "region_events", "region_destroy", "semipar_strerror"):
        assert n in names
    assert sorted(S.SYMBOLS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_record_layouts_match_header():
    from paper_1011_4046_amd.inputs import EVENT_DTYPE, REC_DTYPE
    assert REC_DTYPE.itemsize == 160 and EVENT_DTYPE.itemsize == 56
    assert ctypes.sizeof(S.EvolveParams) == 64
    assert ctypes.sizeof(S.RegionDesc) == 32 + 16 + 32 + 8 + 16
    assert ctypes.sizeof(S.RegionGeom) == 56


def test_argument_errors_without_gpu():
    L = S.lib()
    h = ctypes.c_void_p()
    assert L.region_init_from_surfaces(None, None, 0, ctypes.byref(h)) == -1
    d = S.RegionDesc()
    d.box = -1.0
    assert L.region_init_from_surfaces(ctypes.byref(d), None, 0, ctypes.byref(h)) == -1
    d = S.RegionDesc()
    d.cosmology, d.box = 7, 1.0
    assert L.region_init_from_surfaces(ctypes.byref(d), None, 0, ctypes.byref(h)) == -1
    assert L.region_evolve(None, None, None) == -1
    n = (ctypes.c_int64 * 4)()
    assert L.region_emit_final_surfaces(None, None, None, n, 0) == -1
    L.region_destroy(None)
    assert S.strerror(-2).startswith("inconsistent surface")
    assert "gfx950" in S.version()
