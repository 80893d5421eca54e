"""ctypes binding of the tetrahedral entry points of libfetdpic.so
(include/fetd3.h).

Argument marshalling only: every step of the PIC path runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .fetdpic import PRECISIONS, PUSHERS, FetdError, lib as _base_lib

FIELDS = {"e": 0, "d": 1, "b": 2, "j": 3, "q": 4, "divd": 5, "divb": 6, "edges": 7, "faces": 8,
          "spai_ptr": 9, "spai_col": 10, "spai_val": 11}
STAGES3 = ("faraday", "particles", "ampere", "spmv", "sort")
_DTYPES = {"edges": np.int32, "faces": np.int32, "spai_ptr": np.int32, "spai_col": np.int32}


class MeshDesc3(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("node_xyz", ctypes.c_void_p),
                ("n_tets", ctypes.c_int32), ("tet_nodes", ctypes.c_void_p),
                ("tet_shift", ctypes.c_void_p), ("period", ctypes.c_void_p)]


class Opts3(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("eps0", ctypes.c_double), ("mu0", ctypes.c_double),
                ("c", ctypes.c_double), ("spai_level", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("crossing_cap", ctypes.c_int32), ("resort_every", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class Diag3(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_alive", ctypes.c_int64),
                ("n_lost", ctypes.c_int64), ("n_segments", ctypes.c_int64),
                ("n_nodes", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("n_faces", ctypes.c_int32), ("n_tets", ctypes.c_int32),
                ("gauss_rel", ctypes.c_double), ("divb_rel", ctypes.c_double),
                ("W_E", ctypes.c_double), ("W_B", ctypes.c_double), ("W_kin", ctypes.c_double),
                ("spai_frobenius", ctypes.c_double), ("error_code", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_declared = False


def lib():
    global _declared
    L = _base_lib()
    if not _declared:
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {"fetd3_mesh_create": [P, P, P], "fetd3_fields_set": [P, P, P],
               "fetd3_fields_load": [P, P, P],
               "fetd3_particles_load_bary": [P, D, D, D, I64, P, P, P, P, P],
               "fetd3_pic_step": [P, I32, I32], "fetd3_sort": [P], "fetd3_sync": [P],
               "fetd3_fields_get": [P, I32, P, I64, P],
               "fetd3_particles_get": [P, I32, I64, P, P, P, P, P, P],
               "fetd3_diagnostics": [P, P], "fetd3_profile": [P, I32],
               "fetd3_profile_mask": [P, I32, I32],
               "fetd3_stage_times": [P, P, P]}
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.fetd3_last_error.argtypes = [P]
        L.fetd3_last_error.restype = ctypes.c_char_p
        L.fetd3_destroy.argtypes = [P]
        L.fetd3_destroy.restype = None
        _declared = True
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st, h=None):
    if st != 0:
        msg = lib().fetd3_last_error(h)
        raise FetdError(st, msg.decode() if msg else "")


class Sim3:
    """Owning wrapper of one tetrahedral simulation handle."""

    def __init__(self, mesh, dt, eps0, mu0, c, spai_level=1, device=0, crossing_cap=64,
                 resort_every=20, precision="fp64"):
        xyz = np.ascontiguousarray(mesh.node_xyz, dtype=np.float64)
        tet = np.ascontiguousarray(mesh.tet_nodes, dtype=np.int32)
        sh = None if mesh.tet_shift is None else np.ascontiguousarray(mesh.tet_shift, dtype=np.int8)
        per = None if mesh.period is None else np.ascontiguousarray(mesh.period, dtype=np.float64)
        self._keep = (xyz, tet, sh, per)
        desc = MeshDesc3(xyz.shape[0], _p(xyz), tet.shape[0], _p(tet), _p(sh), _p(per))
        stream = None
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream(device).cuda_stream
        except ImportError:
            pass
        opts = Opts3(float(dt), float(eps0), float(mu0), float(c), int(spai_level), int(device),
                     stream, int(crossing_cap), int(resort_every),
                     PRECISIONS[precision] if isinstance(precision, str) else int(precision))
        h = ctypes.c_void_p()
        _check(lib().fetd3_mesh_create(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(h)))
        self.h = h
        self.n_tets = tet.shape[0]

    def close(self):
        if getattr(self, "h", None):
            lib().fetd3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fields_set(self, b_ext=None, e_ext=None):
        bb = None if b_ext is None else np.ascontiguousarray(b_ext, dtype=np.float64)
        if bb is not None and bb.size == 3:
            bb = np.ascontiguousarray(np.tile(bb.reshape(1, 3), (self.n_tets, 1)))
        ee = None if e_ext is None else np.ascontiguousarray(e_ext, dtype=np.float64)
        _check(lib().fetd3_fields_set(self.h, _p(bb), _p(ee)), self.h)

    def fields_load(self, b=None, d=None):
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
        _check(lib().fetd3_fields_load(self.h, _p(bb), _p(dd)), self.h)

    def load(self, q, m, w, tet, lam, u, slot=None):
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        sl = None if slot is None else np.ascontiguousarray(slot, dtype=np.int8)
        out = ctypes.c_int32()
        _check(lib().fetd3_particles_load_bary(self.h, float(q), float(m), float(w), tet.shape[0],
                                               _p(tet), _p(sl), _p(lam), _p(u),
                                               ctypes.byref(out)), self.h)
        return out.value

    def step(self, n=1, pusher="boris"):
        pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
        _check(lib().fetd3_pic_step(self.h, int(n), pid), self.h)

    def sort(self):
        _check(lib().fetd3_sort(self.h), self.h)

    def sync(self):
        _check(lib().fetd3_sync(self.h), self.h)

    def field(self, which):
        code = FIELDS[which]
        nb = ctypes.c_int64()
        _check(lib().fetd3_fields_get(self.h, code, None, 0, ctypes.byref(nb)), self.h)
        dt = _DTYPES.get(which, np.float64)
        out = np.empty(nb.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().fetd3_fields_get(self.h, code, _p(out), nb.value, ctypes.byref(nb)), self.h)
        return out

    def particles(self, species):
        n = ctypes.c_int64()
        _check(lib().fetd3_particles_get(self.h, int(species), 0, None, None, None, None, None,
                                         ctypes.byref(n)), self.h)
        k = n.value
        tet = np.empty(k, np.int32)
        slot = np.empty(k, np.int8)
        lam = np.empty((k, 3))
        u = np.empty((k, 3))
        pid = np.empty(k, np.int32)
        _check(lib().fetd3_particles_get(self.h, int(species), k, _p(tet), _p(slot), _p(lam),
                                         _p(u), _p(pid), ctypes.byref(n)), self.h)
        return {"tet": tet, "slot": slot, "lam": lam, "u": u, "id": pid}

    def diagnostics(self):
        d = Diag3()
        _check(lib().fetd3_diagnostics(self.h, ctypes.byref(d)), self.h)
        return d.as_dict()

    def profile(self, enable=True, stages=None, every=1):
        """Stage timing on (every stage, or only the named ones of STAGES3;
        on every step, or on steps that are multiples of every) or off."""
        if enable and (stages is not None or every != 1):
            mask = sum(1 << STAGES3.index(k) for k in set(STAGES3 if stages is None else stages))
            _check(lib().fetd3_profile_mask(self.h, mask, int(every)), self.h)
        else:
            _check(lib().fetd3_profile(self.h, 1 if enable else 0), self.h)

    def stage_times(self):
        ms = np.zeros(5)
        n = ctypes.c_int64()
        _check(lib().fetd3_stage_times(self.h, _p(ms), ctypes.byref(n)), self.h)
        return dict(zip(STAGES3, ms)), n.value


def from_workload3(w, spai_level=None, **kw):
    """Create a Sim3 from an inputs3 workload and load its species and applied B."""
    from . import inputs as I
    sim = Sim3(w.mesh, w.dt, I.EPS0, I.MU0, I.C_LIGHT,
               spai_level=w.spai_level if spai_level is None else spai_level, **kw)
    if "b_ext" in w.extra:
        sim.fields_set(b_ext=w.extra["b_ext"])
    for s in w.species:
        sim.load(s.q, s.m, s.w, s.tri, s.lam, s.u)
    return sim
