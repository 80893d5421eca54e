"""The C-ABI library loads and exports every entry point include/fetdpic.h
and include/fetd3.h declare (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(fetd3?_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("fetd_mesh_create", "fetd_particles_load", "fetd_particles_load_bary",
                 "fetd_pic_step", "fetd_fields_get", "fetd_particles_get", "fetd_diagnostics",
                 "fetd_destroy", "fetd_last_error", "fetd_fields_set", "fetd_sync", "fetd_sort",
                 "fetd_info_get", "fetd3_mesh_create", "fetd3_particles_load_bary",
                 "fetd3_pic_step", "fetd3_fields_get", "fetd3_particles_get",
                 "fetd3_diagnostics", "fetd3_destroy"):
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
    assert L.fetd_profile_mask(None, 2, 1) == fetdpic.FETD_E_ARG
    L.fetd_destroy(None)


def test_batch_arguments_without_device():
    """fetd_batch_create refuses an empty list, a null member and a member
    listed twice before it touches any simulation or device."""
    from paper_1707_04333_amd import fetdpic
    L = fetdpic.lib()
    out = ctypes.c_void_p()
    two = (ctypes.c_void_p * 2)(0x1000, 0x1000)  # never dereferenced
    assert L.fetd_batch_create(two, 2, 1, ctypes.byref(out)) == fetdpic.FETD_E_ARG
    assert b"twice" in L.fetd_last_error(None) and not out.value
    null = (ctypes.c_void_p * 2)(0x1000, None)
    assert L.fetd_batch_create(null, 2, 1, ctypes.byref(out)) == fetdpic.FETD_E_ARG
    assert L.fetd_batch_create(two, 0, 1, ctypes.byref(out)) == fetdpic.FETD_E_ARG


def test_mesh_size_limit_without_device():
    """A mesh beyond FETD_MAX_TRIS (the particle kernel's 32-bit table
    offsets) is refused before any array is read or a device is queried."""
    import numpy as np
    from paper_1707_04333_amd import fetdpic
    L = fetdpic.lib()
    xy = np.zeros(6)
    tri = np.zeros(3, np.int32)
    desc = fetdpic.MeshDesc(3, fetdpic._p(xy), fetdpic.MAX_TRIS + 1, fetdpic._p(tri), None, None)
    opts = fetdpic.Opts(0, 1e-12, 8.8e-12, 1.26e-6, 3e8, 1, 0, None, fetdpic.ALLOC_FN(),
                        fetdpic.FREE_FN(), None, 64, 20, 0)
    out = ctypes.c_void_p()
    st = L.fetd_mesh_create(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(out))
    assert st == fetdpic.FETD_E_ARG and not out.value
    assert b"FETD_MAX_TRIS" in L.fetd_last_error(None)


def test_speed_of_light_range_without_device():
    """c^2 outside [1e-250, 1e250] (the range on which the FP64 pushers'
    division by c^2 is correctly rounded) is refused before device work."""
    import numpy as np
    from paper_1707_04333_amd import fetdpic
    L = fetdpic.lib()
    xy = np.array([0.0, 0.0, 1.0, 0.0, 0.0, 1.0])
    tri = np.array([0, 1, 2], np.int32)
    desc = fetdpic.MeshDesc(3, fetdpic._p(xy), 1, fetdpic._p(tri), None, None)
    for c in (1e-126, 1e126, float("inf")):
        opts = fetdpic.Opts(0, 1e-12, 8.8e-12, 1.26e-6, c, 1, 0, None, fetdpic.ALLOC_FN(),
                            fetdpic.FREE_FN(), None, 64, 20, 0)
        out = ctypes.c_void_p()
        st = L.fetd_mesh_create(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(out))
        assert st == fetdpic.FETD_E_ARG and not out.value, c
        assert b"invalid options" in L.fetd_last_error(None)


def test_tet_argument_errors_without_device():
    from paper_1707_04333_amd import fetd3
    L = fetd3.lib()
    out = ctypes.c_void_p()
    assert L.fetd3_mesh_create(None, None, ctypes.byref(out)) == -1
    assert L.fetd3_mesh_create(None, None, None) == -1
    assert b"out is NULL" in L.fetd3_last_error(None)
    assert L.fetd3_pic_step(None, 1, 0) == -1
    assert L.fetd3_profile_mask(None, 2, 1) == -1
    L.fetd3_destroy(None)


def _c_layout(header, structs, tmp_path):
    """sizeof and offsetof of each struct's fields, from the C header as gcc
    lays them out."""
    import subprocess
    lines = [f'#include "{header}"', "#include <stddef.h>", "#include <stdio.h>", "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'    printf("%s %zu\\n", "{cname}", sizeof({cname}));')
        for f in fields:
            lines.append(f'    printf("%s.%s %zu\\n", "{cname}", "{f}", offsetof({cname}, {f}));')
    lines.append("    return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


def test_binding_structs_match_the_headers(tmp_path):
    """Every struct the Python bindings pass through the C-ABI has the size
    and field offsets the public headers give it."""
    from paper_1707_04333_amd import fetd3, fetdpic
    pairs = [("fetdpic.h", [("fetd_mesh_desc", fetdpic.MeshDesc), ("fetd_opts", fetdpic.Opts),
                            ("fetd_info", fetdpic.Info), ("fetd_diag", fetdpic.Diag),
                            ("fetd_tuning", fetdpic.Tuning)]),
             ("fetd3.h", [("fetd3_mesh_desc", fetd3.MeshDesc3), ("fetd3_opts", fetd3.Opts3),
                          ("fetd3_diag", fetd3.Diag3)])]
    renamed = {("fetd3_opts", "stream"): "hip_stream"}  # binding name -> C name
    for header, structs in pairs:
        spec = [(cname, [renamed.get((cname, f), f) for f, _ in py._fields_]) for cname, py in structs]
        got = _c_layout(header, spec, tmp_path)
        for cname, py in structs:
            assert got[cname] == ctypes.sizeof(py), cname
            for f, _ in py._fields_:
                assert got[f"{cname}.{renamed.get((cname, f), f)}"] == getattr(py, f).offset, (cname, f)
