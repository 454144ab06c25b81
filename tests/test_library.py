"""CPU checks of the C-ABI library: it loads without a GPU and exports every
entry point that include/gaborfields.h declares; argument validation that
happens before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gaborfields.h")
LIB = os.path.join(ROOT, "paper_2602_05081_amd", "libgaborfields.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gf_status|uint64_t|const char\*)\s+(gf_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        from paper_2602_05081_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(so):
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_every_entry_point():
    from paper_2602_05081_amd import _lib
    assert set(declared()) <= set(_lib.exported_symbols())


def test_lod_cells_host_only(so):
    so.gf_mask_lod_cells.restype = ctypes.c_uint64
    assert so.gf_mask_lod_cells(0) == 0xFFF
    assert so.gf_mask_lod_cells(3) == 0x7


def test_null_arguments_rejected_without_device(so):
    so.gf_scene_create.restype = ctypes.c_int
    so.gf_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    assert so.gf_scene_create(None, ctypes.c_int64(10), None, None, ctypes.byref(out)) == -1
    assert b"NULL" in so.gf_last_error()
