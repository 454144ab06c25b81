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


def _desc(**kw):
    from paper_2602_05081_amd import _lib
    d = _lib.render_desc(spp=2, stochastic=True)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,msg", [("level_strategy", 9, b"level strategy"),
                                             ("bin_strategy", -1, b"bin strategy"),
                                             ("beta", 1.0, b"beta"), ("delta", 1.5, b"delta"),
                                             ("free_flight", 2, b"free_flight"), ("spp", 0, b"spp")])
def test_render_description_validated_on_the_host(so, field, value, msg):
    """An invalid render description is rejected by the size query and by
    the camera render before anything touches a device."""
    from paper_2602_05081_amd import _lib
    L = _lib.lib()
    cam = _lib.camera(1, width=16, height=16)
    d = _desc(**{field: value})
    size = ctypes.c_size_t()
    assert L.gf_render_workspace_size(None, ctypes.byref(cam), ctypes.byref(d), ctypes.byref(size)) == -1
    assert msg in L.gf_last_error()
    assert L.gf_render(None, ctypes.byref(cam), ctypes.byref(d), None, 0, None, None, None) == -1
    assert msg in L.gf_last_error()


def test_render_camera_validated_on_the_host(so):
    from paper_2602_05081_amd import _lib
    L = _lib.lib()
    d = _desc()
    size = ctypes.c_size_t()
    for cam in (_lib.camera(1, width=0, height=16), _lib.camera(3, width=8, height=8),
                _lib.camera(1, eye=(0.5, 0.5, 0.5), target=(0.5, 0.5, 0.5))):
        assert L.gf_render_workspace_size(None, ctypes.byref(cam), ctypes.byref(d), ctypes.byref(size)) == -1
    # a valid description and camera with no scene: NULL argument
    cam = _lib.camera(1, width=16, height=16)
    assert L.gf_render_workspace_size(None, ctypes.byref(cam), ctypes.byref(d), ctypes.byref(size)) == -1
    assert b"NULL" in L.gf_last_error()
