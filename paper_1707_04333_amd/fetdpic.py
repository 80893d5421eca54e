"""ctypes binding of libfetdpic.so (include/fetdpic.h).

Argument marshalling only: every step of the PIC path runs in the library's
HIP kernels.  PyTorch, when present, supplies device memory (its caching
allocator, through the alloc/free callbacks of fetd_opts) and the stream.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfetdpic.so")

FETD_OK, FETD_E_ARG, FETD_E_MESH, FETD_E_OOM, FETD_E_HIP, FETD_E_TRACK, FETD_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
PUSHERS = {"boris": 0, "boris_tan": 1, "vay": 2, "hc": 3}
PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_f64field": 2}
MAX_SPECIES_PARTICLES = (1 << 28) - 1024
MAX_TRIS = 1 << 26
FIELDS = {"e": 0, "d": 1, "b": 2, "j": 3, "q": 4, "spai_ptr": 5, "spai_col": 6, "spai_val": 7,
          "edges": 8, "tri_edge": 9, "divd": 10}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class FetdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fetdpic status {status}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("node_xy", ctypes.c_void_p),
                ("n_tris", ctypes.c_int32), ("tri_nodes", ctypes.c_void_p),
                ("tri_shift", ctypes.c_void_p), ("period", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("dt", ctypes.c_double),
                ("eps0", ctypes.c_double), ("mu0", ctypes.c_double), ("c", ctypes.c_double),
                ("spai_level", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", ctypes.c_void_p), ("crossing_cap", ctypes.c_int32),
                ("resort_every", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("record_crossings", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("n_edges", ctypes.c_int32), ("n_free_edges", ctypes.c_int32),
                ("n_free_nodes", ctypes.c_int32), ("spai_nnz", ctypes.c_int64),
                ("spai_frobenius", ctypes.c_double), ("n_species", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_alive", ctypes.c_int64),
                ("n_lost", ctypes.c_int64), ("n_segments", ctypes.c_int64),
                ("gauss_abs", ctypes.c_double), ("gauss_rel", ctypes.c_double),
                ("dce_abs", ctypes.c_double), ("dce_rel", ctypes.c_double),
                ("W_E", ctypes.c_double), ("W_B", ctypes.c_double), ("W_kin", ctypes.c_double),
                ("error_code", ctypes.c_int32), ("error_particle", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_1707_04333_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.fetd_mesh_create.argtypes = [P, P, P]
        L.fetd_fields_set.argtypes = [P, P, P, P]
        L.fetd_particles_load_bary.argtypes = [P, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int64, P, P, P, P, P]
        L.fetd_particles_load.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int64, P, P, P, P]
        L.fetd_pic_step.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
        L.fetd_sort.argtypes = [P]
        L.fetd_sync.argtypes = [P]
        L.fetd_fields_get.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64, P]
        L.fetd_particles_get.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P]
        L.fetd_diagnostics.argtypes = [P, P]
        L.fetd_info_get.argtypes = [P, P]
        L.fetd_last_error.argtypes = [P]
        L.fetd_last_error.restype = ctypes.c_char_p
        optional = {"fetd_profile": [P, ctypes.c_int32], "fetd_stage_times": [P, P, P],
                    "fetd_profile_mask": [P, ctypes.c_int32, ctypes.c_int32],
                    "fetd_autotune": [P, ctypes.c_int32, ctypes.c_int32, P],
                    "fetd_set_tile": [P, ctypes.c_int32],
                    "fetd_get_tile": [P, P],
                    "fetd_set_scan": [P, ctypes.c_int32],
                    "fetd_set_defer_exits": [P, ctypes.c_int32],
                    "fetd_get_defer_exits": [P, P],
                    "fetd_crossings_get": [P, ctypes.c_int32, ctypes.c_int64, P, P, P],
                    "fetd_get_scan": [P, P],
                    "fetd_set_resort": [P, ctypes.c_int32],
                    "fetd_batch_create": [P, ctypes.c_int32, ctypes.c_int32, P],
                    "fetd_batch_step": [P, ctypes.c_int32, ctypes.c_int32],
                    "fetd_batch_stats": [P, P, P, P],
                    "fetd_copy_ceiling": [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P],
                    "fetd_batch_step_noalloc": [P, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32],
                    "fetd_set_absorber": [P, P],
                    "fetd_set_pml": [P, P, ctypes.c_int32],
                    "fetd_set_ext_scale": [P, ctypes.c_double],
                    "fetd_probe_set": [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int64],
                    "fetd_probe_get": [P, P, ctypes.c_int64, P],
                    "fetd_fields_load": [P, P, P]}
        for name, args in optional.items():
            if hasattr(L, name):
                getattr(L, name).argtypes = args
                getattr(L, name).restype = ctypes.c_int
        if hasattr(L, "fetd_batch_destroy"):
            L.fetd_batch_destroy.argtypes = [P]
            L.fetd_batch_destroy.restype = None
        L.fetd_destroy.argtypes = [P]
        L.fetd_destroy.restype = None
        for name in ("fetd_mesh_create", "fetd_fields_set", "fetd_particles_load_bary",
                     "fetd_particles_load", "fetd_pic_step", "fetd_sort", "fetd_sync",
                     "fetd_fields_get", "fetd_particles_get", "fetd_diagnostics",
                     "fetd_info_get"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st, sim=None):
    if st != FETD_OK:
        msg = lib().fetd_last_error(sim)
        raise FetdError(st, msg.decode() if msg else "")


class _TorchMemory:
    """Device memory from torch's caching allocator on the current stream."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)

    def _do_alloc(self, nbytes, user):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                                self.stream))
        except Exception:
            return None

    def _do_free(self, ptr, user):
        # at interpreter shutdown torch may already be torn down; the
        # process exit releases the device memory then
        cuda = getattr(getattr(self.torch, "cuda", None), "caching_allocator_delete", None)
        if ptr and cuda is not None:
            cuda(int(ptr))


# ---------------------------------------------------------------------------
# Entry points with the C-ABI's names.
# ---------------------------------------------------------------------------

def mesh_create(mesh, dt, eps0, mu0, c, precision="fp64", spai_level=1, device=0,
                crossing_cap=64, resort_every=20, deterministic=False, record_crossings=0,
                use_torch=True):
    """fetd_mesh_create.  ``mesh`` has node_xy, tri_nodes, tri_shift, period."""
    node_xy = np.ascontiguousarray(mesh.node_xy, dtype=np.float64)
    tri = np.ascontiguousarray(mesh.tri_nodes, dtype=np.int32)
    shift = None if mesh.tri_shift is None else np.ascontiguousarray(mesh.tri_shift, dtype=np.int8)
    period = None if mesh.period is None else np.ascontiguousarray(mesh.period, dtype=np.float64)
    desc = MeshDesc(node_xy.shape[0], _p(node_xy), tri.shape[0], _p(tri), _p(shift), _p(period))
    mem = None
    stream = None
    if use_torch:
        try:
            import torch
            if torch.cuda.is_available():
                mem = _TorchMemory(device)
                stream = mem.stream.cuda_stream
        except ImportError:
            mem = None
    opts = Opts(PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                float(dt), float(eps0), float(mu0), float(c), int(spai_level), int(device),
                stream, mem._alloc if mem else ALLOC_FN(), mem._free if mem else FREE_FN(), None,
                int(crossing_cap), int(resort_every), 1 if deterministic else 0,
                int(record_crossings))
    h = ctypes.c_void_p()
    _check(lib().fetd_mesh_create(ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(h)))
    return h, mem


def fields_set(h, bz_ext=None, e_ext=None, e_affine=None):
    bz = None if bz_ext is None else np.ascontiguousarray(bz_ext, dtype=np.float64)
    ee = None if e_ext is None else np.ascontiguousarray(e_ext, dtype=np.float64)
    af = None if e_affine is None else np.ascontiguousarray(e_affine, dtype=np.float64)
    _check(lib().fetd_fields_set(h, _p(bz), _p(ee), _p(af)), h)


def set_absorber(h, sigma_tri):
    sg = None if sigma_tri is None else np.ascontiguousarray(sigma_tri, dtype=np.float64)
    _check(lib().fetd_set_absorber(h, _p(sg)), h)


def set_pml(h, sigma_tri, axis=0):
    sg = None if sigma_tri is None else np.ascontiguousarray(sigma_tri, dtype=np.float64)
    _check(lib().fetd_set_pml(h, _p(sg), int(axis)), h)


def fields_load(h, b=None, d=None):
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    _check(lib().fetd_fields_load(h, _p(bb), _p(dd)), h)


def set_ext_scale(h, scale):
    _check(lib().fetd_set_ext_scale(h, float(scale)), h)


def probe_set(h, xy, every=1, max_samples=1):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    _check(lib().fetd_probe_set(h, xy.shape[0], _p(xy), int(every), int(max_samples)), h)


def probe_get(h, n_points):
    ns = ctypes.c_int64()
    _check(lib().fetd_probe_get(h, None, 0, ctypes.byref(ns)), h)
    out = np.empty((ns.value, n_points, 2))
    _check(lib().fetd_probe_get(h, _p(out), out.nbytes, ctypes.byref(ns)), h)
    return out


def particles_load_bary(h, q, m, w, tri, lam, u, slot=None):
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    sl = None if slot is None else np.ascontiguousarray(slot, dtype=np.int8)
    out = ctypes.c_int32()
    _check(lib().fetd_particles_load_bary(h, q, m, w, tri.shape[0], _p(tri), _p(sl), _p(lam),
                                          _p(u), ctypes.byref(out)), h)
    return out.value


def particles_load(h, q, m, w, xy, u, tri_hint=None):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    th = None if tri_hint is None else np.ascontiguousarray(tri_hint, dtype=np.int32)
    out = ctypes.c_int32()
    _check(lib().fetd_particles_load(h, q, m, w, xy.shape[0], _p(xy), _p(u), _p(th),
                                     ctypes.byref(out)), h)
    return out.value


def pic_step(h, n_steps, pusher="boris"):
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    _check(lib().fetd_pic_step(h, int(n_steps), pid), h)


def sort(h):
    _check(lib().fetd_sort(h), h)


def sync(h):
    _check(lib().fetd_sync(h), h)


def fields_get(h, which):
    sel = FIELDS[which] if isinstance(which, str) else int(which)
    nbytes = ctypes.c_int64()
    _check(lib().fetd_fields_get(h, sel, None, 0, ctypes.byref(nbytes)), h)
    dtype = np.int32 if sel in (5, 6, 8, 9) else np.float64
    out = np.empty(nbytes.value // np.dtype(dtype).itemsize, dtype=dtype)
    _check(lib().fetd_fields_get(h, sel, _p(out), out.nbytes, ctypes.byref(nbytes)), h)
    return out


def particles_get(h, species):
    n = ctypes.c_int64()
    st = lib().fetd_particles_get(h, int(species), 0, None, None, None, None, None,
                                  ctypes.byref(n))
    if st not in (FETD_OK, FETD_E_ARG):
        _check(st, h)
    cnt = n.value
    tri = np.empty(cnt, dtype=np.int32)
    slot = np.empty(cnt, dtype=np.int8)
    lam = np.empty((cnt, 2))
    u = np.empty((cnt, 2))
    ids = np.empty(cnt, dtype=np.int64)
    _check(lib().fetd_particles_get(h, int(species), cnt, _p(tri), _p(slot), _p(lam), _p(u),
                                    _p(ids), ctypes.byref(n)), h)
    return dict(tri=tri, slot=slot, lam=lam, u=u, id=ids)


def crossings_get(h, species, record):
    """fetd_crossings_get: (count [n], tris [n, record]) of the last step, in
    the order of particles_get."""
    n = ctypes.c_int64()
    st = lib().fetd_crossings_get(h, int(species), 0, None, None, ctypes.byref(n))
    if st not in (FETD_OK, FETD_E_ARG):
        _check(st, h)
    cnt = n.value
    count = np.empty(cnt, dtype=np.int32)
    tris = np.empty((cnt, int(record)), dtype=np.int32)
    _check(lib().fetd_crossings_get(h, int(species), cnt, _p(count), _p(tris), ctypes.byref(n)),
           h)
    return count, tris


def diagnostics(h):
    d = Diag()
    _check(lib().fetd_diagnostics(h, ctypes.byref(d)), h)
    return d.as_dict()


def info(h):
    i = Info()
    _check(lib().fetd_info_get(h, ctypes.byref(i)), h)
    return {k: getattr(i, k) for k, _ in i._fields_}


STAGES = ("faraday", "particles", "ampere", "spmv", "sort")


AUTOTUNE_CANDIDATES = (5, 10, 20, 40, 80, 160)
TILE_CANDIDATES = (512, 768, 1024, 1280, 1536, 1792, 2048)
SCAN_CANDIDATES = (64, 16, 8)


class Tuning(ctypes.Structure):
    _fields_ = [("resort_every", ctypes.c_int32), ("tile_particles", ctypes.c_int32),
                ("scan_lanes", ctypes.c_int32), ("defer_exits", ctypes.c_int32),
                ("resort_cost_ms", ctypes.c_double * 6),
                ("tile_cost_ms", ctypes.c_double * 7), ("scan_cost_ms", ctypes.c_double * 3),
                ("defer_cost_ms", ctypes.c_double * 2)]


def autotune(h, pusher="boris", trial_steps=160, with_costs=False):
    """fetd_autotune: tunes the tile, the scan group width, the exit mode
    (FP32 particles), then the re-sort interval.  Returns the chosen re-sort
    interval; with_costs, a dict with the choices ("resort_every", "tile",
    "scan", "defer_exits") and the measured cost in ms per step of every
    candidate tried ("costs", "tile_costs", "scan_costs", "defer_costs")."""
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    t = Tuning()
    _check(lib().fetd_autotune(h, pid, int(trial_steps), ctypes.byref(t)), h)
    if not with_costs:
        return t.resort_every
    return {"resort_every": t.resort_every, "tile": t.tile_particles, "scan": t.scan_lanes,
            "defer_exits": t.defer_exits,
            "costs": {c: float(v) for c, v in zip(AUTOTUNE_CANDIDATES, t.resort_cost_ms)
                      if v >= 0},
            "tile_costs": {c: float(v) for c, v in zip(TILE_CANDIDATES, t.tile_cost_ms)},
            "scan_costs": {c: float(v) for c, v in zip(SCAN_CANDIDATES, t.scan_cost_ms)},
            "defer_costs": {c: float(v) for c, v in enumerate(t.defer_cost_ms) if v >= 0}}


def set_defer_exits(h, on):
    _check(lib().fetd_set_defer_exits(h, int(on)), h)


def get_defer_exits(h):
    out = ctypes.c_int32()
    _check(lib().fetd_get_defer_exits(h, ctypes.byref(out)), h)
    return out.value


def set_tile(h, tile_particles):
    _check(lib().fetd_set_tile(h, int(tile_particles)), h)


def get_tile(h):
    out = ctypes.c_int32()
    _check(lib().fetd_get_tile(h, ctypes.byref(out)), h)
    return out.value


def set_scan(h, lanes):
    _check(lib().fetd_set_scan(h, int(lanes)), h)


def get_scan(h):
    out = ctypes.c_int32()
    _check(lib().fetd_get_scan(h, ctypes.byref(out)), h)
    return out.value


def set_resort(h, every):
    _check(lib().fetd_set_resort(h, int(every)), h)


def stage_mask(stages):
    """Bit mask of stage names (STAGES) for fetd_profile_mask."""
    return sum(1 << STAGES.index(k) for k in set(stages))


def profile(h, enable=True, stages=None, every=1):
    """Stage timing on (every stage, or only the named ones; on every
    step, or on steps that are multiples of every) or off."""
    if enable and (stages is not None or every != 1):
        mask = stage_mask(STAGES if stages is None else stages)
        _check(lib().fetd_profile_mask(h, mask, int(every)), h)
    else:
        _check(lib().fetd_profile(h, 1 if enable else 0), h)


def stage_times(h):
    ms = np.zeros(len(STAGES))
    n = np.zeros(len(STAGES), dtype=np.int64)
    _check(lib().fetd_stage_times(h, _p(ms), _p(n)), h)
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}


def copy_ceiling(device=0, nbytes=1 << 30, reps=5):
    """fetd_copy_ceiling: measured copy bandwidth (read + write) in GB/s."""
    out = ctypes.c_double()
    _check(lib().fetd_copy_ceiling(int(device), int(nbytes), int(reps), ctypes.byref(out)))
    return out.value


def destroy(h):
    lib().fetd_destroy(h)


class Sim:
    """Owning wrapper: one simulation handle and the memory callbacks it
    needs kept alive."""

    def __init__(self, mesh, dt, eps0, mu0, c, **kw):
        self.record = int(kw.get("record_crossings", 0))
        self.h, self._mem = mesh_create(mesh, dt, eps0, mu0, c, **kw)

    def close(self):
        if self.h:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fields_set(self, **kw):
        fields_set(self.h, **kw)

    def set_absorber(self, sigma_tri):
        set_absorber(self.h, sigma_tri)

    def set_pml(self, sigma_tri, axis=0):
        set_pml(self.h, sigma_tri, axis)

    def set_ext_scale(self, scale):
        set_ext_scale(self.h, scale)

    def fields_load(self, b=None, d=None):
        fields_load(self.h, b, d)

    def probe_set(self, xy, every=1, max_samples=1):
        self._probe_n = 0 if xy is None else np.asarray(xy).reshape(-1, 2).shape[0]
        probe_set(self.h, np.zeros((0, 2)) if xy is None else xy, every, max_samples)

    def probe_get(self):
        return probe_get(self.h, getattr(self, "_probe_n", 0))

    def load(self, q, m, w, tri, lam, u, slot=None):
        return particles_load_bary(self.h, q, m, w, tri, lam, u, slot)

    def load_xy(self, q, m, w, xy, u, tri_hint=None):
        return particles_load(self.h, q, m, w, xy, u, tri_hint)

    def step(self, n=1, pusher="boris"):
        pic_step(self.h, n, pusher)

    def sort(self):
        sort(self.h)

    def sync(self):
        sync(self.h)

    def field(self, which):
        return fields_get(self.h, which)

    def particles(self, species):
        return particles_get(self.h, species)

    def crossings(self, species):
        return crossings_get(self.h, species, self.record)

    def diagnostics(self):
        return diagnostics(self.h)

    def info(self):
        return info(self.h)

    def profile(self, enable=True, stages=None, every=1):
        profile(self.h, enable, stages, every)

    def autotune(self, pusher="boris", trial_steps=160, with_costs=False):
        return autotune(self.h, pusher, trial_steps, with_costs)

    def set_resort(self, every):
        set_resort(self.h, every)

    def set_defer_exits(self, on):
        set_defer_exits(self.h, on)

    def get_defer_exits(self):
        return get_defer_exits(self.h)

    def set_tile(self, tile_particles):
        set_tile(self.h, tile_particles)

    def get_tile(self):
        return get_tile(self.h)

    def set_scan(self, lanes):
        set_scan(self.h, lanes)

    def get_scan(self):
        return get_scan(self.h)

    def stage_times(self):
        return stage_times(self.h)


def batch_create(sims, use_graph=True):
    """fetd_batch_create over a list of Sim objects (same device, stream,
    precision)."""
    arr = (ctypes.c_void_p * len(sims))(*[sm.h.value for sm in sims])
    h = ctypes.c_void_p()
    _check(lib().fetd_batch_create(arr, len(sims), 1 if use_graph else 0, ctypes.byref(h)))
    return h


def batch_step(b, n_steps, pusher="boris"):
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    _check(lib().fetd_batch_step(b, int(n_steps), pid))


def batch_stats(b):
    """(graph captures, graph replays, eager steps) of a batch."""
    c, r, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fetd_batch_stats(b, ctypes.byref(c), ctypes.byref(r), ctypes.byref(e)))
    return {"graph_captures": c.value, "graph_replays": r.value, "eager_steps": e.value}


def batch_step_noalloc(sims, n_steps, pusher="boris"):
    """fetd_batch_step_noalloc over a list of Sim objects."""
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    arr = (ctypes.c_void_p * len(sims))(*[sm.h.value for sm in sims])
    _check(lib().fetd_batch_step_noalloc(arr, len(sims), int(n_steps), pid))


def batch_destroy(b):
    lib().fetd_batch_destroy(b)


class Batch:
    """Owning wrapper of a batch; keeps its member Sims alive."""

    def __init__(self, sims, use_graph=True):
        self.sims = list(sims)
        self.h = batch_create(self.sims, use_graph)

    def step(self, n=1, pusher="boris"):
        batch_step(self.h, n, pusher)

    def stats(self):
        return batch_stats(self.h)

    def close(self):
        if self.h:
            batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, precision=None, **kw):
    """Create a Sim from an inputs.Workload and load its species and fields."""
    from . import inputs as I
    sim = Sim(w.mesh, w.dt, I.EPS0, I.MU0, w.extra.get("c", I.C_LIGHT),
              precision=precision or w.precision, spai_level=kw.pop("spai_level", w.spai_level),
              **kw)
    bz = w.extra.get("bz_tri")
    if bz is None and w.bz_ext:
        bz = np.full(w.mesh.n_tris, float(w.bz_ext))
    if bz is not None or w.e_affine is not None:
        sim.fields_set(bz_ext=bz, e_affine=w.e_affine)
    if "sigma_tri" in w.extra:
        sim.set_absorber(w.extra["sigma_tri"])
    for s in w.species:
        sim.load(s.q, s.m, s.w, s.tri, s.lam, s.u)
    return sim
