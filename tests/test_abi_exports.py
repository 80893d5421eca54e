"""The C-ABI library loads and exports every entry point include/fetdpic.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fetdpic.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fetd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("fetd_mesh_create", "fetd_particles_load", "fetd_particles_load_bary",
                 "fetd_pic_step", "fetd_fields_get", "fetd_particles_get", "fetd_diagnostics",
                 "fetd_destroy", "fetd_last_error", "fetd_fields_set", "fetd_sync", "fetd_sort",
                 "fetd_info_get"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_1707_04333_amd import fetdpic
    lib = ctypes.CDLL(fetdpic.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_argument_errors_without_device():
    """Argument validation happens before any device call."""
    from paper_1707_04333_amd import fetdpic
    L = fetdpic.lib()
    out = ctypes.c_void_p()
    assert L.fetd_mesh_create(None, None, ctypes.byref(out)) == fetdpic.FETD_E_ARG
    assert L.fetd_mesh_create(None, None, None) == fetdpic.FETD_E_ARG
    assert b"out is NULL" in L.fetd_last_error(None)
    assert L.fetd_pic_step(None, 1, 0) == fetdpic.FETD_E_ARG
    L.fetd_destroy(None)
