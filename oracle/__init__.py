"""FP64 CPU oracle of the relativistic charge-conserving FETD-PIC step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the library.  It
shares no code with the HIP library (``paper_1707_04333_amd``).

Setup (mesh topology, geometry, Hodge matrices, inverse) is plain numpy;
the per-step particle and field arithmetic is plain single-threaded C in
``fetd_oracle.c`` (built by ``build()`` below with ``-ffp-contract=off``).

Paper: Na, Moon, Omelchenko, Teixeira, arXiv:1707.04333.  Sections cited
as "Sec. II.A" (field update, eqs. semi.dis.curl.1/2 and semi.dis.div.1/2),
"Sec. II.B" (gather), "Sec. II.C" (particle update and pushers),
"Sec. II.D" (scatter, eqs. scatter.charge.assign, I.assign, full.dis.cont).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

BORIS, BORIS_TAN, VAY, HC = 0, 1, 2, 3
PUSHERS = {"boris": BORIS, "boris_tan": BORIS_TAN, "vay": VAY, "hc": HC}


def build(force: bool = True) -> str:
    """Compile fetd_oracle.c (triangles) and fetd3_oracle.c (tetrahedra)
    into liboracle.so (plain C, FP64, no FMA)."""
    srcs = [os.path.join(_HERE, "fetd_oracle.c"), os.path.join(_HERE, "fetd3_oracle.c")]
    newest = max(os.path.getmtime(s) for s in srcs)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


class OMesh(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int32), ("ne", ctypes.c_int32), ("nn", ctypes.c_int32),
                ("tri_node", ctypes.c_void_p), ("tri_edge", ctypes.c_void_p),
                ("tri_sign", ctypes.c_void_p), ("tri_nbr", ctypes.c_void_p),
                ("tri_nbrk", ctypes.c_void_p), ("vxy", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("area", ctypes.c_void_p),
                ("edge_tri", ctypes.c_void_p), ("edge_tsign", ctypes.c_void_p),
                ("edge_free", ctypes.c_void_p), ("mt_ptr", ctypes.c_void_p),
                ("mt_col", ctypes.c_void_p), ("mt_val", ctypes.c_void_p)]


def _declare(L):
    P = ctypes.c_void_p
    L.o_push.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, P]
    L.o_push.restype = None
    L.o_gather_e.argtypes = [P, P, P, ctypes.c_int, P, P]
    L.o_gather_e.restype = None
    L.o_move.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P,
                         ctypes.c_int, P, P, P]
    L.o_move.restype = ctypes.c_int
    L.o_faraday.argtypes = [P, P, P, ctypes.c_double, P, P]
    L.o_faraday.restype = None
    L.o_ampere.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    L.o_ampere.restype = None
    L.o_particles.argtypes = [P, P, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int64, P, P, P, P, P,
                              P, P, P, ctypes.c_int, P]
    L.o_particles.restype = ctypes.c_int
    L.o_particles_omp.argtypes = [ctypes.c_int] + L.o_particles.argtypes
    L.o_particles_omp.restype = ctypes.c_int
    L.o_charge.argtypes = [P, ctypes.c_double, ctypes.c_int64, P, P, P, P]
    L.o_charge.restype = None
    L.o_spai.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, ctypes.c_int64]
    L.o_spai.restype = ctypes.c_int64
    L.o_ampere_pml.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P,
                               P, P, P, P, P, P, P, P, P, P, P]
    L.o_ampere_pml.restype = None


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# ---------------------------------------------------------------------------
# Mesh topology and geometry (Sec. II.A: incidence matrices C, S and the
# dual incidences C~ = C^T, S~ = S^T; entries in {-1, 0, 1}).
# ---------------------------------------------------------------------------

class Topology:
    """Edges, incidence, neighbours and Whitney-form geometry of a
    triangle mesh.  Edges are node pairs oriented low -> high global id and
    numbered in lexicographic (low, high) order."""

    def __init__(self, node_xy, tri_nodes, tri_shift=None, period=None):
        tri = np.ascontiguousarray(tri_nodes, dtype=np.int32)
        nf = tri.shape[0]
        nn = node_xy.shape[0]
        v = node_xy[tri].astype(np.float64)
        if tri_shift is not None:
            v = v + tri_shift.astype(np.float64) * np.asarray(period, dtype=np.float64)[None, None, :]
        # local edge k joins local nodes a=(k+1)%3 -> b=(k+2)%3
        a = tri[:, [1, 2, 0]]
        b = tri[:, [2, 0, 1]]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        if np.any(lo == hi):
            raise ValueError("degenerate edge (mesh too small for its periodicity)")
        pairs = np.stack([lo.reshape(-1), hi.reshape(-1)], axis=1)
        uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        ne = uniq.shape[0]
        self.nf, self.ne, self.nn = nf, ne, nn
        self.tri_node = tri
        self.edge_lo = uniq[:, 0].astype(np.int32)
        self.edge_hi = uniq[:, 1].astype(np.int32)
        self.tri_edge = inv.reshape(nf, 3).astype(np.int32)
        self.tri_sign = np.where(a < b, 1, -1).astype(np.int8)
        # edge -> adjacent (triangle, local k)
        occ_t = np.repeat(np.arange(nf, dtype=np.int32), 3)
        occ_k = np.tile(np.arange(3, dtype=np.int32), nf)
        order = np.argsort(inv, kind="stable")
        counts = np.bincount(inv, minlength=ne)
        if counts.max() > 2:
            raise ValueError("non-manifold mesh: an edge has more than two triangles")
        start = np.concatenate([[0], np.cumsum(counts)])
        et = np.full((ne, 2), -1, dtype=np.int32)
        ek = np.full((ne, 2), -1, dtype=np.int32)
        et[:, 0] = occ_t[order[start[:-1]]]
        ek[:, 0] = occ_k[order[start[:-1]]]
        two = counts == 2
        et[two, 1] = occ_t[order[start[:-1][two] + 1]]
        ek[two, 1] = occ_k[order[start[:-1][two] + 1]]
        self.edge_tri = et
        self.edge_tsign = np.zeros((ne, 2), dtype=np.int8)
        for j in range(2):
            ok = et[:, j] >= 0
            self.edge_tsign[ok, j] = self.tri_sign[et[ok, j], ek[ok, j]]
        nbr = np.full((nf, 3), -1, dtype=np.int32)
        nbk = np.full((nf, 3), -1, dtype=np.int8)
        nbr[et[two, 0], ek[two, 0]] = et[two, 1]
        nbk[et[two, 0], ek[two, 0]] = ek[two, 1]
        nbr[et[two, 1], ek[two, 1]] = et[two, 0]
        nbk[et[two, 1], ek[two, 1]] = ek[two, 0]
        self.tri_nbr = nbr
        self.tri_nbrk = nbk
        self.edge_free = two.astype(np.uint8)  # one-sided edges lie on the PEC wall
        node_free = np.ones(nn, dtype=np.uint8)
        node_free[self.edge_lo[~two]] = 0
        node_free[self.edge_hi[~two]] = 0
        self.node_free = node_free
        # Geometry: A2 = 2A from vertex 0; grad l_k = perp(x_b - x_a) / A2.
        self.vxy = np.ascontiguousarray(v.reshape(nf, 6))
        x = v[:, :, 0]
        y = v[:, :, 1]
        a2 = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
        if np.any(a2 <= 0):
            raise ValueError("triangles must be counter-clockwise with positive area")
        self.area = 0.5 * a2
        g = np.empty((nf, 3, 2))
        for k in range(3):
            ia, ib = (k + 1) % 3, (k + 2) % 3
            g[:, k, 0] = -(y[:, ib] - y[:, ia]) / a2
            g[:, k, 1] = (x[:, ib] - x[:, ia]) / a2
        self.grad = np.ascontiguousarray(g.reshape(nf, 6))

    def curl_matrix(self):
        """Dense-free incidence C (faces x edges) as (rows, cols, vals)."""
        r = np.repeat(np.arange(self.nf), 3)
        return r, self.tri_edge.reshape(-1), self.tri_sign.reshape(-1).astype(np.int64)

    def grad_matrix(self):
        """Incidence G (edges x nodes): -1 at the low node, +1 at the high."""
        r = np.repeat(np.arange(self.ne), 2)
        c = np.stack([self.edge_lo, self.edge_hi], axis=1).reshape(-1)
        v = np.tile(np.array([-1, 1], dtype=np.int64), self.ne)
        return r, c, v

    def divergence(self, x_edge):
        """S~ x = -G^T x: net outflow of an edge quantity at every node
        (Sec. II.D, eq. full.dis.cont)."""
        out = np.zeros(self.nn)
        np.add.at(out, self.edge_lo, x_edge)
        np.add.at(out, self.edge_hi, -x_edge)
        return out


def hodge_eps(T: Topology, eps0: float):
    """[*eps]_ij = eps0 * int W1_i . W1_j (Sec. II.A), assembled from the
    element integrals int l_a l_b = A (1 + delta_ab) / 12.  Rows and columns
    of wall (non-free) edges are replaced by the identity.  Returns CSR
    (ptr, col, val) with sorted columns."""
    nf = T.nf
    G = T.grad.reshape(nf, 3, 2)
    A = T.area
    rows, cols, vals = [], [], []
    for k in range(3):
        a, b = (k + 1) % 3, (k + 2) % 3
        for l in range(3):
            c, d = (l + 1) % 3, (l + 2) % 3

            def I(i, j):
                return A * (2.0 if i == j else 1.0) / 12.0

            def gd(i, j):
                return G[:, i, 0] * G[:, j, 0] + G[:, i, 1] * G[:, j, 1]

            val = (gd(b, d) * I(a, c) - gd(b, c) * I(a, d)
                   - gd(a, d) * I(b, c) + gd(a, c) * I(b, d))
            val = eps0 * T.tri_sign[:, k] * T.tri_sign[:, l] * val
            rows.append(T.tri_edge[:, k])
            cols.append(T.tri_edge[:, l])
            vals.append(val)
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals)
    free = T.edge_free.astype(bool)
    keep = free[r] & free[c]
    r, c, v = r[keep], c[keep], v[keep]
    wall = np.nonzero(~free)[0]
    r = np.concatenate([r, wall])
    c = np.concatenate([c, wall])
    v = np.concatenate([v, np.ones(wall.size)])
    return _coo_to_csr(T.ne, r, c, v)


def hodge_eps_parts(T: Topology, eps0: float):
    """The two parts of [*eps] (Sec. II.A) carried by the x and the y
    components of the Whitney 1-forms: eps0 int W_i,x W_j,x and
    eps0 int W_i,y W_j,y, assembled like hodge_eps (their sum is [*eps] on
    the free edges).  Returns two CSR triples; wall rows are empty."""
    nf = T.nf
    G = T.grad.reshape(nf, 3, 2)
    A = T.area
    free = T.edge_free.astype(bool)
    out = []
    for comp in (0, 1):
        rows, cols, vals = [], [], []
        for k in range(3):
            a, b = (k + 1) % 3, (k + 2) % 3
            for l in range(3):
                c, d = (l + 1) % 3, (l + 2) % 3

                def I(i, j):
                    return A * (2.0 if i == j else 1.0) / 12.0

                def gd(i, j):
                    return G[:, i, comp] * G[:, j, comp]

                val = (gd(b, d) * I(a, c) - gd(b, c) * I(a, d)
                       - gd(a, d) * I(b, c) + gd(a, c) * I(b, d))
                rows.append(T.tri_edge[:, k])
                cols.append(T.tri_edge[:, l])
                vals.append(eps0 * T.tri_sign[:, k] * T.tri_sign[:, l] * val)
        r = np.concatenate(rows).astype(np.int64)
        c = np.concatenate(cols).astype(np.int64)
        v = np.concatenate(vals)
        keep = free[r] & free[c]
        out.append(_coo_to_csr(T.ne, r[keep], c[keep], v[keep]))
    return out


def pml_setup(T: Topology, sigma_tri, dt: float, eps0: float, axis: int = 0):
    """Uniaxial PML stretched along `axis` (0: layers normal to x, 1: to y)
    with conductivity sigma_tri per triangle: the PML rows (free edges whose
    conductivity, the mean of their triangles', is positive), kappa =
    sigma/eps0 per row, the rows of the normal and tangential parts of
    [*eps], zeroed auxiliary fluxes, and the matched magnetic loss factor
    per triangle (as absorber_damp)."""
    sg = np.asarray(sigma_tri, dtype=np.float64)
    f0, f1 = T.edge_tri[:, 0], T.edge_tri[:, 1]
    se = sg[f0].copy()
    two = f1 >= 0
    se[two] = 0.5 * (sg[f0[two]] + sg[f1[two]])
    rows = np.nonzero((se > 0) & T.edge_free.astype(bool))[0].astype(np.int32)
    parts = hodge_eps_parts(T, eps0)
    Mn, Mt = parts[axis], parts[1 - axis]

    def take(Mx):
        ptr, col, val = Mx
        cnt = ptr[rows + 1] - ptr[rows]
        optr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
        idx = np.concatenate([np.arange(ptr[r], ptr[r + 1]) for r in rows]) if rows.size else \
            np.zeros(0, np.int64)
        return optr, col[idx].astype(np.int32), val[idx].copy()

    xt = sg * dt / (2.0 * eps0)
    damp_b = np.where(sg > 0, (1.0 - xt) / (1.0 + xt), 1.0)
    return {"rows": rows, "kappa": se[rows] / eps0, "n": take(Mn), "t": take(Mt),
            "psi": np.zeros(rows.size), "phi": np.zeros(rows.size), "extra": np.zeros(T.ne),
            "damp_b": damp_b, "axis": axis}


def _coo_to_csr(n, r, c, v):
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    key = r * n + c
    first = np.concatenate([[True], key[1:] != key[:-1]])
    idx = np.cumsum(first) - 1
    vs = np.zeros(int(first.sum()))
    np.add.at(vs, idx, v)
    r, c = r[first], c[first]
    ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(ptr, r + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int32)
    return ptr, c.astype(np.int32), vs


def csr_to_dense(n, ptr, col, val):
    out = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(ptr))
    out[rows, col] = val
    return out


def csr_matvec(ptr, col, val, x):
    rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    out = np.zeros(ptr.size - 1)
    np.add.at(out, rows, val * x[col])
    return out


def approx_inverse(T: Topology, Meps, level: int):
    """Approximate inverse M~ of [*eps] (Sec. II.A): level >= 0 is the
    Frobenius SPAI on the pattern of the level-th power of the graph of
    [*eps] (level 0: diagonal), symmetrised; level -1 is the exact inverse
    (dense; small meshes only)."""
    ptr, col, val = Meps
    n = T.ne
    if level < 0:
        dense = np.linalg.inv(csr_to_dense(n, ptr, col, val))
        dense = 0.5 * (dense + dense.T)
        rr, cc = np.nonzero(np.ones((n, n), dtype=bool))
        return _coo_to_csr(n, rr, cc, dense[rr, cc])
    cap = int(n) * 64
    optr = np.zeros(n + 1, dtype=np.int32)
    ocol = np.zeros(cap, dtype=np.int32)
    oval = np.zeros(cap)
    nnz = lib().o_spai(n, _p(ptr), _p(col), _p(val), level, _p(optr), _p(ocol), _p(oval), cap)
    if nnz < 0:
        raise RuntimeError("SPAI pattern too large")
    return optr, ocol[:nnz].copy(), oval[:nnz].copy()


# ---------------------------------------------------------------------------
# Simulation driver
# ---------------------------------------------------------------------------

class OSpecies:
    def __init__(self, q, m, w, tri, lam, u, slot=None):
        self.q, self.m, self.w = float(q), float(m), float(w)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32).copy()
        self.lam = np.ascontiguousarray(lam, dtype=np.float64).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).copy()
        n = self.tri.shape[0]
        self.slot = (np.zeros(n, dtype=np.int8) if slot is None
                     else np.ascontiguousarray(slot, dtype=np.int8).copy())

    @property
    def n(self):
        return self.tri.shape[0]


class OracleSim:
    """One PIC run: the four procedures of Sec. II in the order field
    update (Faraday half), gather, push, scatter, field update (Ampere
    half):  b^{n+1/2} = b^{n-1/2} - dt C e^n; particles gather e^n and
    B^n = (B^{n+1/2} + B^{n-1/2})/2, push u^{n-1/2} -> u^{n+1/2}, move and
    deposit i^{n+1/2}; d^{n+1} = d^n + dt (C^T [*mu^-1] b^{n+1/2} - i^{n+1/2}),
    e^{n+1} = M~ d^{n+1}."""

    def __init__(self, mesh, dt, species, eps0, mu0, c, spai_level=1, bz_ext=None,
                 e_ext=None, affine=None, cap=64, damp=None, damp_b=None, pml=None):
        self.T = Topology(mesh.node_xy, mesh.tri_nodes, mesh.tri_shift, mesh.period) \
            if not isinstance(mesh, Topology) else mesh
        T = self.T
        self.dt, self.eps0, self.mu0, self.c = float(dt), float(eps0), float(mu0), float(c)
        self.Meps = hodge_eps(T, eps0)
        self.Mt = approx_inverse(T, self.Meps, spai_level)
        self.b = np.zeros(T.nf)
        self.d = np.zeros(T.ne)
        self.e = np.zeros(T.ne)
        self.cur = np.zeros(T.ne)
        self.last_cur = np.zeros(T.ne)
        if bz_ext is not None and np.ndim(bz_ext) == 0:
            bz_ext = np.full(T.nf, float(bz_ext))
        self.bz_ext = None if bz_ext is None else np.ascontiguousarray(bz_ext, dtype=np.float64)
        self.e_ext = None if e_ext is None else np.ascontiguousarray(e_ext, dtype=np.float64)
        self.affine = None if affine is None else np.ascontiguousarray(affine, dtype=np.float64)
        self.damp = None if damp is None else np.ascontiguousarray(damp, dtype=np.float64)
        self.damp_b = None if damp_b is None else np.ascontiguousarray(damp_b, dtype=np.float64)
        self.species = [OSpecies(*s) if not isinstance(s, OSpecies) else s for s in species]
        self.pml = pml  # pml_setup() record, or None
        self.cap = cap
        self.step_count = 0
        self.segments = 0
        self.lost = 0
        self._keep = []
        self._mesh_struct()

    def _mesh_struct(self):
        T = self.T
        ptr, col, val = self.Mt
        arrs = dict(tri_node=T.tri_node, tri_edge=T.tri_edge, tri_sign=T.tri_sign,
                    tri_nbr=T.tri_nbr, tri_nbrk=T.tri_nbrk, vxy=T.vxy, grad=T.grad,
                    area=T.area, edge_tri=T.edge_tri, edge_tsign=T.edge_tsign,
                    edge_free=T.edge_free, mt_ptr=ptr, mt_col=col, mt_val=val)
        self._keep = {k: np.ascontiguousarray(v) for k, v in arrs.items()}
        self.ms = OMesh(T.nf, T.ne, T.nn, *[_p(self._keep[k]) for k in
                                            ["tri_node", "tri_edge", "tri_sign", "tri_nbr",
                                             "tri_nbrk", "vxy", "grad", "area", "edge_tri",
                                             "edge_tsign", "edge_free", "mt_ptr", "mt_col",
                                             "mt_val"]])

    def step(self, n_steps=1, pusher="boris", threads=1, record=0):
        """n_steps steps with the given pusher.  threads > 1 runs the
        particle stage on that many OpenMP threads (the timing mode:
        contiguous chunks of particles, private currents added in thread
        order); the default single thread is the parity mode.  record > 0
        keeps, per species, the triangles of the first `record` straight
        pieces of every particle's last move (s.seq [n, record], -1 beyond
        the pieces) and the number of pieces (s.nseq [n])."""
        L = lib()
        pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
        ms = ctypes.byref(self.ms)
        for _ in range(n_steps):
            b_new = np.empty_like(self.b)
            L.o_faraday(ms, _p(self.b), _p(self.e), self.dt, _p(self.damp_b), _p(b_new))
            counts = np.zeros(2, dtype=np.int64)
            bad = np.zeros(1, dtype=np.int64)
            for s in self.species:
                if record > 0:
                    s.seq = np.full((s.n, record), -1, dtype=np.int32)
                    s.nseq = np.zeros(s.n, dtype=np.int32)
                args = (ms, _p(self.e), _p(self.e_ext), _p(self.b), _p(b_new),
                        _p(self.bz_ext), _p(self.affine), pid, s.q, s.m, s.w,
                        self.dt, self.c, self.cap, s.n, _p(s.tri), _p(s.slot),
                        _p(s.lam), _p(s.u), _p(self.cur), _p(counts), _p(bad),
                        _p(s.seq) if record > 0 else None, int(record),
                        _p(s.nseq) if record > 0 else None)
                if threads > 1:
                    rc = L.o_particles_omp(int(threads), *args)
                else:
                    rc = L.o_particles(*args)
                if rc != 0:
                    raise RuntimeError(f"oracle particle stage failed rc={rc} at particle {bad[0]}")
            if self.pml is not None:
                P = self.pml
                L.o_ampere_pml(ms, _p(b_new), _p(self.cur), self.dt, self.mu0,
                               int(P["rows"].size), _p(P["rows"]), _p(P["kappa"]),
                               _p(P["n"][0]), _p(P["n"][1]), _p(P["n"][2]),
                               _p(P["t"][0]), _p(P["t"][1]), _p(P["t"][2]),
                               _p(P["psi"]), _p(P["phi"]), _p(P["extra"]), _p(self.d),
                               _p(self.e))
            else:
                L.o_ampere(ms, _p(b_new), _p(self.cur), self.dt, self.mu0, _p(self.damp),
                           _p(self.d), _p(self.e))
            self.b = b_new
            self.last_cur[:] = self.cur
            self.cur[:] = 0.0
            self.segments += int(counts[0])
            self.lost += int(counts[1])
            self.step_count += 1

    # ---- diagnostics (Sec. II.A eq. semi.dis.div.2, Sec. II.D) ----
    def charge(self):
        qn = np.zeros(self.T.nn)
        for s in self.species:
            lib().o_charge(ctypes.byref(self.ms), s.q * s.w, s.n, _p(s.tri), _p(s.slot),
                           _p(s.lam), _p(qn))
        return qn

    def gauss_lhs(self):
        """S~ [*eps] e, evaluated as S~ d (d = [*eps]-effective flux)."""
        return self.T.divergence(self.d)

    def positions(self, s):
        """Cartesian positions (image frame of each triangle)."""
        T = self.T
        L = np.empty((s.n, 3))
        for r in range(3):
            sel = s.slot == r
            p, q = (r + 1) % 3, (r + 2) % 3
            L[sel, p] = s.lam[sel, 0]
            L[sel, q] = s.lam[sel, 1]
            L[sel, r] = (1.0 - s.lam[sel, 0]) - s.lam[sel, 1]
        v = T.vxy[np.maximum(s.tri, 0)].reshape(-1, 3, 2)
        return np.einsum("nk,nkd->nd", L, v)

    def energies(self):
        ptr, col, val = self.Meps
        WE = 0.5 * float(self.e @ csr_matvec(ptr, col, val, self.e))
        WB = 0.5 * float(np.sum(self.b * self.b / (self.mu0 * self.T.area)))
        WK = 0.0
        for s in self.species:
            ok = s.tri >= 0
            g = np.sqrt(1.0 + np.sum(s.u[ok] ** 2, axis=1) / self.c ** 2)
            WK += float(np.sum(s.w * s.m * self.c ** 2 * (g - 1.0)))
        return WE, WB, WK


def absorber_damp(T: Topology, sigma_tri, dt: float, eps0: float):
    """Losses of the absorbing layer (the build's own stand-in for the
    paper's PML).  Electric: edge conductivity = mean over its triangles; d
    is multiplied by (1 - x)/(1 + x), x = sigma dt/(2 eps0), after each
    Ampere update.  Magnetic: the matched loss sigma_m = sigma mu0/eps0 on
    each triangle, so b is multiplied by the same factor of its own sigma
    after each Faraday update; with both, a plane wave entering the layer
    at normal incidence meets no impedance step (Z = sqrt(mu0/eps0) for
    any sigma).  Returns (damp per edge, damp per triangle, nodes kept in
    the Gauss residual)."""
    sg = np.asarray(sigma_tri, dtype=np.float64)
    f0, f1 = T.edge_tri[:, 0], T.edge_tri[:, 1]
    se = sg[f0].copy()
    two = f1 >= 0
    se[two] = 0.5 * (sg[f0[two]] + sg[f1[two]])
    x = se * dt / (2.0 * eps0)
    damp = np.where(se > 0, (1.0 - x) / (1.0 + x), 1.0)
    xt = sg * dt / (2.0 * eps0)
    damp_b = np.where(sg > 0, (1.0 - xt) / (1.0 + xt), 1.0)
    keep = T.node_free.astype(bool).copy()
    lossy = se > 0
    keep[T.edge_lo[lossy]] = False
    keep[T.edge_hi[lossy]] = False
    return damp, damp_b, keep


def push(pusher, u, E, B, q, m, dt, c):
    """Single 3-D momentum update through the oracle pusher."""
    alpha = q * dt / (2.0 * m)
    u = np.ascontiguousarray(u, dtype=np.float64)
    eps = np.ascontiguousarray(np.asarray(E, dtype=np.float64) * alpha)
    beta = np.ascontiguousarray(np.asarray(B, dtype=np.float64) * alpha)
    out = np.zeros(3)
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    lib().o_push(pid, _p(u), _p(eps), _p(beta), c, _p(out))
    return out


def push_raw(pusher, u, eps, beta, c):
    u = np.ascontiguousarray(u, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros(3)
    pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
    lib().o_push(pid, _p(u), _p(eps), _p(beta), c, _p(out))
    return out


def move_one(sim: OracleSim, tri, slot, pair, dx, dy, qdt=1.0, cap=64):
    """Track one particle through the mesh without touching the
    simulation's current; returns (tri, slot, pair, lost, segments, cur)
    with segments a list of (triangle, L_start[3], L_end[3])."""
    t = np.array([tri], dtype=np.int32)
    s = np.array([slot], dtype=np.int8)
    pr = np.ascontiguousarray(pair, dtype=np.float64).copy()
    cur = np.zeros(sim.T.ne)
    lost = np.zeros(1, dtype=np.int32)
    st = np.zeros(cap, dtype=np.int32)
    sl = np.zeros(cap * 6)
    ns = lib().o_move(ctypes.byref(sim.ms), _p(t), _p(s), _p(pr), float(dx), float(dy),
                      float(qdt), _p(cur), cap, _p(lost), _p(st), _p(sl))
    if ns < 0:
        raise RuntimeError("crossing cap exceeded")
    segs = [(int(st[i]), sl[6 * i:6 * i + 3].copy(), sl[6 * i + 3:6 * i + 6].copy())
            for i in range(ns)]
    return int(t[0]), int(s[0]), pr, bool(lost[0]), segs, cur


def gather_e(sim: OracleSim, tri, L, e=None):
    E = np.zeros(3)
    e = sim.e if e is None else np.ascontiguousarray(e, dtype=np.float64)
    Lc = np.ascontiguousarray(L, dtype=np.float64)
    lib().o_gather_e(ctypes.byref(sim.ms), _p(e), None, int(tri), _p(Lc), _p(E))
    return E[:2]
