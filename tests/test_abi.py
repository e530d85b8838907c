"""Host-side checks of the C ABI: the library builds for gfx950, loads without a
GPU and exports every function include/wgeo.h declares (no compute calls)."""
import ctypes
import os
import re

from paper_2609_20964_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "wgeo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("wg_recon_forward", "wg_recon_backward", "wg_sample_sdf_normals", "wg_submit", "wg_poll"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(_lib.LIB_PATH), "build libwgeo.so first"
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding covers the same set
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_struct_layouts_match_header_sizes():
    # sizes implied by include/wgeo.h on x86-64
    assert ctypes.sizeof(_lib.WgGrid) == 12 + 4 + 24 + 8
    assert ctypes.sizeof(_lib.WgSolveOpts) == 8 + 5 * 4 + 4   # + tail padding to 8
    assert ctypes.sizeof(_lib.WgStats) == 4 + 4 + 8 + 8 + 8 + 8 + 4 + 32 + 4 + 8


def test_footprint_is_a_host_computation():
    L = _lib.lib()
    g = _lib.make_grid(64)
    fp = L.wg_recon_footprint(ctypes.byref(g), 100000)
    assert fp > 64 ** 3 * 40
    g256 = _lib.make_grid(256)
    assert L.wg_recon_footprint(ctypes.byref(g256), 300000) > 8 * fp
