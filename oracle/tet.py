"""FP64 CPU oracle of the FETD-PIC step on tetrahedra (Sec. II in three
dimensions: Whitney 1-forms on edges, 2-forms on faces, incidence C of
faces x edges and S of cells x faces, Hodge matrices on edges and faces).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Setup is numpy; the
per-step arithmetic is the C of ``fetd3_oracle.c``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import PUSHERS, _coo_to_csr, _p, csr_matvec, lib

LE = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]])
LF = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])


class O3Mesh(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("ne", ctypes.c_int32), ("nf", ctypes.c_int32),
                ("nn", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in (
                    "tet_node", "tet_edge", "tet_esign", "tet_face", "tet_fpar", "tet_nbr",
                    "tet_nbrmap", "grad", "vxyz", "face_edge", "face_esign", "edge_free",
                    "mnu_ptr", "mnu_col", "mnu_val", "mt_ptr", "mt_col", "mt_val")]


def _declare3(L):
    P = ctypes.c_void_p
    if getattr(L, "_o3_declared", False):
        return
    L.o3_gather_e.argtypes = [P, P, P, ctypes.c_int, P, P]
    L.o3_gather_e.restype = None
    L.o3_gather_b.argtypes = [P, P, ctypes.c_int, P, P]
    L.o3_gather_b.restype = None
    L.o3_move.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, P, ctypes.c_int, P]
    L.o3_move.restype = ctypes.c_int
    L.o3_faraday.argtypes = [P, P, P, ctypes.c_double, P]
    L.o3_faraday.restype = None
    L.o3_ampere.argtypes = [P, P, P, ctypes.c_double, P, P, P]
    L.o3_ampere.restype = None
    L.o3_particles.argtypes = [P, P, P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int64, P, P, P, P, P, P, P, P]
    L.o3_particles.restype = ctypes.c_int
    L.o3_charge.argtypes = [P, ctypes.c_double, ctypes.c_int64, P, P, P, P]
    L.o3_charge.restype = None
    L._o3_declared = True


def lib3():
    L = lib()
    _declare3(L)
    return L


class Topology3:
    """Edges, faces, incidence, neighbours and Whitney geometry of a
    tetrahedral mesh.  Edges are node pairs (low, high) and faces sorted
    node triples, both numbered in lexicographic order."""

    def __init__(self, node_xyz, tet_nodes, tet_shift=None, period=None):
        tet = np.ascontiguousarray(tet_nodes, dtype=np.int32)
        nt, nn = tet.shape[0], node_xyz.shape[0]
        v = node_xyz[tet].astype(np.float64)
        if tet_shift is not None:
            v = v + tet_shift.astype(np.float64) * np.asarray(period, dtype=np.float64)[None, None, :]
        self.nt, self.nn = nt, nn
        self.tet_node = tet
        # edges
        a, b = tet[:, LE[:, 0]], tet[:, LE[:, 1]]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        if np.any(lo == hi):
            raise ValueError("degenerate edge (mesh too small for its periodicity)")
        uniq, inv = np.unique(np.stack([lo.ravel(), hi.ravel()], 1), axis=0, return_inverse=True)
        self.ne = uniq.shape[0]
        self.edge_lo = uniq[:, 0].astype(np.int32)
        self.edge_hi = uniq[:, 1].astype(np.int32)
        self.tet_edge = inv.reshape(nt, 6).astype(np.int32)
        self.tet_esign = np.where(a < b, 1, -1).astype(np.int8)
        # faces: sorted global triples
        fl = tet[:, LF]                                   # [nt, 4, 3] local sorted order
        fs = np.sort(fl, axis=2)
        if np.any(fs[:, :, 0] == fs[:, :, 1]) or np.any(fs[:, :, 1] == fs[:, :, 2]):
            raise ValueError("degenerate face")
        funiq, finv = np.unique(fs.reshape(-1, 3), axis=0, return_inverse=True)
        self.nf = funiq.shape[0]
        self.face_node = funiq.astype(np.int32)
        self.tet_face = finv.reshape(nt, 4).astype(np.int32)
        # parity of the local sorted order against the global sorted order
        order = np.argsort(fl, axis=2)                    # positions of the global order
        par = np.ones((nt, 4), dtype=np.int8)
        for x, y in ((0, 1), (0, 2), (1, 2)):
            par = np.where(order[:, :, x] > order[:, :, y], -par, par).astype(np.int8)
        self.tet_fpar = par
        # geometry
        J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("tetrahedra must be positively oriented")
        self.vol = det / 6.0
        Ji = np.linalg.inv(J)                             # rows: grad l_1..l_3
        g = np.empty((nt, 4, 3))
        g[:, 1:, :] = Ji
        g[:, 0, :] = -Ji.sum(axis=1)
        self.grad = np.ascontiguousarray(g.reshape(nt, 12))
        self.vxyz = np.ascontiguousarray(v.reshape(nt, 12))
        # outward sign of each global face in its tetrahedron: the global
        # normal is fpar times the local sorted normal, which is outward for
        # k even and inward for k odd in a positive tetrahedron; checked
        # against geometry below
        loc_out = np.array([1, -1, 1, -1], dtype=np.int8)
        self.tet_fout = (par * loc_out[None, :]).astype(np.int8)
        nrm = np.cross(v[:, LF[:, 1]] - v[:, LF[:, 0]], v[:, LF[:, 2]] - v[:, LF[:, 0]])
        outward = -g  # grad l_k points into the tetrahedron, towards node k
        chk = np.sign(np.einsum("tkx,tkx->tk", nrm, outward)).astype(np.int8)
        if not np.array_equal(chk, loc_out[None, :].repeat(nt, 0)):
            raise ValueError("face orientation check failed")
        # faces -> tetrahedra, neighbours and node maps
        occ_t = np.repeat(np.arange(nt, dtype=np.int32), 4)
        occ_k = np.tile(np.arange(4, dtype=np.int32), nt)
        fo = np.argsort(finv, kind="stable")
        cnt = np.bincount(finv, minlength=self.nf)
        if cnt.max() > 2:
            raise ValueError("non-manifold mesh: a face has more than two tetrahedra")
        st = np.concatenate([[0], np.cumsum(cnt)])
        ft = np.full((self.nf, 2), -1, dtype=np.int32)
        fk = np.full((self.nf, 2), -1, dtype=np.int32)
        ft[:, 0] = occ_t[fo[st[:-1]]]
        fk[:, 0] = occ_k[fo[st[:-1]]]
        two = cnt == 2
        ft[two, 1] = occ_t[fo[st[:-1][two] + 1]]
        fk[two, 1] = occ_k[fo[st[:-1][two] + 1]]
        self.face_tet, self.face_tk = ft, fk
        nbr = np.full((nt, 4), -1, dtype=np.int32)
        nbmap = np.full((nt, 4, 4), -1, dtype=np.int8)
        for s0, s1 in ((0, 1), (1, 0)):
            t0, k0 = ft[two, s0], fk[two, s0]
            t1, k1 = ft[two, s1], fk[two, s1]
            nbr[t0, k0] = t1
            for j in range(4):
                gj = tet[t0, j]
                hit = np.full(t0.shape[0], -1, dtype=np.int8)
                for jj in range(4):
                    hit = np.where(tet[t1, jj] == gj, jj, hit).astype(np.int8)
                sel = j != k0
                nbmap[t0[sel], k0[sel], j] = hit[sel]
            nbmap[t0, k0, k0] = k1
        if np.any((nbr >= 0)[:, :, None] & (nbmap < 0)):
            raise ValueError("neighbour node map incomplete")
        self.tet_nbr = nbr
        self.tet_nbrmap = np.ascontiguousarray(nbmap.reshape(nt, 16))
        # C: global face (i<j<l) bounds i->j (+1), j->l (+1), l->i (-1)
        fn = self.face_node
        ekey = {(int(x), int(y)): i for i, (x, y) in enumerate(uniq)}
        fe = np.empty((self.nf, 3), dtype=np.int32)
        for f in range(self.nf):
            i, j, l = fn[f]
            fe[f] = (ekey[(i, j)], ekey[(j, l)], ekey[(i, l)])
        self.face_edge = fe
        self.face_esign = np.tile(np.array([1, 1, -1], dtype=np.int8), (self.nf, 1))
        # boundary (PEC): one-sided faces, their edges and nodes are not free
        bf = ~two
        self.face_free = two.astype(np.uint8)
        ef = np.ones(self.ne, dtype=np.uint8)
        ef[fe[bf].ravel()] = 0
        self.edge_free = ef
        nf_ = np.ones(nn, dtype=np.uint8)
        nf_[fn[bf].ravel()] = 0
        self.node_free = nf_

    def curl(self, e):
        """C e: circulation of an edge quantity around every face."""
        return np.sum(self.face_esign * e[self.face_edge], axis=1)

    def face_divergence(self, b):
        """S b: net outward flux of a face quantity from every tetrahedron
        (Sec. II.A, eq. semi.dis.div.1)."""
        return np.sum(self.tet_fout * b[self.tet_face], axis=1)

    def divergence(self, x_edge):
        """S~ x = -G^T x: net outflow of an edge quantity at every node."""
        out = np.zeros(self.nn)
        np.add.at(out, self.edge_lo, x_edge)
        np.add.at(out, self.edge_hi, -x_edge)
        return out


def _mass(vol, p, q):
    """int l_p l_q over a tetrahedron = V (1 + delta_pq) / 20."""
    return vol * (2.0 if p == q else 1.0) / 20.0


def hodge_eps3(T: Topology3, eps0: float):
    """[*eps]_ij = eps0 int W1_i . W1_j, wall rows/columns replaced by the
    identity; CSR (ptr, col, val)."""
    G = T.grad.reshape(T.nt, 4, 3)
    rows, cols, vals = [], [], []
    for k in range(6):
        a, b = LE[k]
        for l in range(6):
            c, d = LE[l]

            def gd(i, j):
                return np.einsum("tx,tx->t", G[:, i], G[:, j])

            val = (gd(b, d) * _mass(T.vol, a, c) - gd(b, c) * _mass(T.vol, a, d)
                   - gd(a, d) * _mass(T.vol, b, c) + gd(a, c) * _mass(T.vol, b, d))
            rows.append(T.tet_edge[:, k])
            cols.append(T.tet_edge[:, l])
            vals.append(eps0 * T.tet_esign[:, k] * T.tet_esign[:, l] * val)
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals)
    free = T.edge_free.astype(bool)
    keep = free[r] & free[c]
    wall = np.nonzero(~free)[0]
    return _coo_to_csr(T.ne, np.concatenate([r[keep], wall]), np.concatenate([c[keep], wall]),
                       np.concatenate([v[keep], np.ones(wall.size)]))


def whitney2_coeffs(T: Topology3):
    """Y[t, k, n]: W2 of local face k (local sorted order) = 2 sum_n l_n
    Y[t, k, n] with Y = grad l_q x grad l_r for n = p etc. (cyclic), 0 for
    the node opposite the face."""
    G = T.grad.reshape(T.nt, 4, 3)
    Y = np.zeros((T.nt, 4, 4, 3))
    for k in range(4):
        p, q, r = LF[k]
        Y[:, k, p] = np.cross(G[:, q], G[:, r])
        Y[:, k, q] = np.cross(G[:, r], G[:, p])
        Y[:, k, r] = np.cross(G[:, p], G[:, q])
    return Y


def hodge_nu3(T: Topology3, mu0: float):
    """[*mu^-1]_fg = (1/mu0) int W2_f . W2_g over the mesh (faces); CSR."""
    Y = whitney2_coeffs(T)
    rows, cols, vals = [], [], []
    for k in range(4):
        for l in range(4):
            acc = np.zeros(T.nt)
            for p in range(4):
                for q in range(4):
                    acc += _mass(T.vol, p, q) * np.einsum("tx,tx->t", Y[:, k, p], Y[:, l, q])
            rows.append(T.tet_face[:, k])
            cols.append(T.tet_face[:, l])
            vals.append(4.0 * T.tet_fpar[:, k] * T.tet_fpar[:, l] * acc / mu0)
    return _coo_to_csr(T.nf, np.concatenate(rows).astype(np.int64),
                       np.concatenate(cols).astype(np.int64), np.concatenate(vals))


def approx_inverse3(T: Topology3, Meps, level: int):
    """Frobenius SPAI of [*eps] on the level-th power of its graph,
    symmetrised (the same construction as for triangles)."""
    ptr, col, val = Meps
    n = T.ne
    if level < 0:
        from . import csr_to_dense
        dense = np.linalg.inv(csr_to_dense(n, ptr, col, val))
        dense = 0.5 * (dense + dense.T)
        rr, cc = np.nonzero(np.ones((n, n), dtype=bool))
        return _coo_to_csr(n, rr, cc, dense[rr, cc])
    cap = int(n) * 256
    optr = np.zeros(n + 1, dtype=np.int32)
    ocol = np.zeros(cap, dtype=np.int32)
    oval = np.zeros(cap)
    nnz = lib().o_spai(n, _p(ptr), _p(col), _p(val), level, _p(optr), _p(ocol), _p(oval), cap)
    if nnz < 0:
        raise RuntimeError("SPAI pattern too large")
    return optr, ocol[:nnz].copy(), oval[:nnz].copy()


class OSpecies3:
    def __init__(self, q, m, w, tet, lam, u, slot=None):
        self.q, self.m, self.w = float(q), float(m), float(w)
        self.tet = np.ascontiguousarray(tet, dtype=np.int32).copy()
        self.lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1, 3).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3).copy()
        n = self.tet.shape[0]
        self.slot = (np.zeros(n, dtype=np.int8) if slot is None
                     else np.ascontiguousarray(slot, dtype=np.int8).copy())

    @property
    def n(self):
        return self.tet.shape[0]


class OracleSim3:
    """One PIC run on tetrahedra, in the order of Sec. II: b^{n+1/2} =
    b^{n-1/2} - dt C e^n; gather E^n, B^n = (B^{n+1/2} + B^{n-1/2})/2 at
    r^n; push; move and deposit i^{n+1/2}; d^{n+1} = d^n + dt (C^T
    [*mu^-1] b^{n+1/2} - i^{n+1/2}), e^{n+1} = M~ d^{n+1}."""

    def __init__(self, mesh, dt, species, eps0, mu0, c, spai_level=1, b_ext=None, e_ext=None,
                 cap=64):
        self.T = mesh if isinstance(mesh, Topology3) else Topology3(
            mesh.node_xyz, mesh.tet_nodes, mesh.tet_shift, mesh.period)
        T = self.T
        self.dt, self.eps0, self.mu0, self.c = float(dt), float(eps0), float(mu0), float(c)
        self.Meps = hodge_eps3(T, eps0)
        self.Mnu = hodge_nu3(T, mu0)
        self.Mt = approx_inverse3(T, self.Meps, spai_level)
        self.b = np.zeros(T.nf)
        self.d = np.zeros(T.ne)
        self.e = np.zeros(T.ne)
        self.cur = np.zeros(T.ne)
        self.last_cur = np.zeros(T.ne)
        if b_ext is not None:
            b_ext = np.asarray(b_ext, dtype=np.float64)
            if b_ext.ndim == 1:
                b_ext = np.tile(b_ext, (T.nt, 1))
            b_ext = np.ascontiguousarray(b_ext.reshape(-1))
        self.b_ext = b_ext
        self.e_ext = None if e_ext is None else np.ascontiguousarray(e_ext, dtype=np.float64)
        self.species = [s if isinstance(s, OSpecies3) else OSpecies3(*s) for s in species]
        self.cap = cap
        self.step_count = self.segments = self.lost = 0
        self._work = np.zeros(T.nf + T.ne)
        self._bavg = np.zeros(T.nf)
        keep = dict(tet_node=T.tet_node, tet_edge=T.tet_edge, tet_esign=T.tet_esign,
                    tet_face=T.tet_face, tet_fpar=T.tet_fpar, tet_nbr=T.tet_nbr,
                    tet_nbrmap=T.tet_nbrmap, grad=T.grad, vxyz=T.vxyz,
                    face_edge=np.ascontiguousarray(T.face_edge),
                    face_esign=np.ascontiguousarray(T.face_esign), edge_free=T.edge_free,
                    mnu_ptr=self.Mnu[0], mnu_col=self.Mnu[1], mnu_val=self.Mnu[2],
                    mt_ptr=self.Mt[0], mt_col=self.Mt[1], mt_val=self.Mt[2])
        self._keep = {k: np.ascontiguousarray(v) for k, v in keep.items()}
        self.ms = O3Mesh(T.nt, T.ne, T.nf, T.nn, *[_p(self._keep[k]) for k, _ in
                                                   O3Mesh._fields_[4:]])

    def step(self, n_steps=1, pusher="boris"):
        L = lib3()
        pid = PUSHERS[pusher] if isinstance(pusher, str) else int(pusher)
        ms = ctypes.byref(self.ms)
        for _ in range(n_steps):
            b_new = np.empty_like(self.b)
            L.o3_faraday(ms, _p(self.b), _p(self.e), self.dt, _p(b_new))
            counts = np.zeros(2, dtype=np.int64)
            bad = np.zeros(1, dtype=np.int64)
            for s in self.species:
                rc = L.o3_particles(ms, _p(self.e), _p(self.e_ext), _p(self.b), _p(b_new),
                                    _p(self.b_ext), pid, s.q, s.m, s.w, self.dt, self.c, self.cap,
                                    s.n, _p(s.tet), _p(s.slot), _p(s.lam), _p(s.u), _p(self.cur),
                                    _p(self._bavg), _p(counts), _p(bad))
                if rc != 0:
                    raise RuntimeError(f"oracle particle stage failed rc={rc} at {bad[0]}")
            L.o3_ampere(ms, _p(b_new), _p(self.cur), self.dt, _p(self.d), _p(self.e),
                        _p(self._work))
            self.b = b_new
            self.last_cur[:] = self.cur
            self.cur[:] = 0.0
            self.segments += int(counts[0])
            self.lost += int(counts[1])
            self.step_count += 1

    def charge(self):
        qn = np.zeros(self.T.nn)
        for s in self.species:
            lib3().o3_charge(ctypes.byref(self.ms), s.q * s.w, s.n, _p(s.tet), _p(s.slot),
                             _p(s.lam), _p(qn))
        return qn

    def lambdas(self, s):
        """Four barycentrics per particle from the stored triple and slot."""
        L = np.empty((s.n, 4))
        for r in range(4):
            sel = s.slot == r
            L[sel, (r + 1) % 4] = s.lam[sel, 0]
            L[sel, (r + 2) % 4] = s.lam[sel, 1]
            L[sel, (r + 3) % 4] = s.lam[sel, 2]
            L[sel, r] = ((1.0 - s.lam[sel, 0]) - s.lam[sel, 1]) - s.lam[sel, 2]
        return L

    def positions(self, s):
        v = self.T.vxyz[np.maximum(s.tet, 0)].reshape(-1, 4, 3)
        return np.einsum("nk,nkd->nd", self.lambdas(s), v)

    def energies(self):
        WE = 0.5 * float(self.e @ csr_matvec(*self.Meps, self.e))
        WB = 0.5 * float(self.b @ csr_matvec(*self.Mnu, self.b))
        WK = 0.0
        for s in self.species:
            ok = s.tet >= 0
            g = np.sqrt(1.0 + np.sum(s.u[ok] ** 2, axis=1) / self.c ** 2)
            WK += float(np.sum(s.w * s.m * self.c ** 2 * (g - 1.0)))
        return WE, WB, WK


def gather3(sim: OracleSim3, tet, L, e=None, b=None):
    """E and B (from face fluxes b, default the current b) at barycentrics L
    (4 values) in tetrahedron tet."""
    Lc = np.ascontiguousarray(L, dtype=np.float64)
    E = np.zeros(3)
    B = np.zeros(3)
    ee = sim.e if e is None else np.ascontiguousarray(e, dtype=np.float64)
    bb = sim.b if b is None else np.ascontiguousarray(b, dtype=np.float64)
    lib3().o3_gather_e(ctypes.byref(sim.ms), _p(ee), None, int(tet), _p(Lc), _p(E))
    lib3().o3_gather_b(ctypes.byref(sim.ms), _p(bb), int(tet), _p(Lc), _p(B))
    return E, B


def move3(sim: OracleSim3, tet, slot, s3, dr, qdt=1.0, cap=64):
    """Move one particle; returns (tet, slot, stored triple, lost, pieces,
    current vector)."""
    cur = np.zeros(sim.T.ne)
    t = ctypes.c_int32(int(tet))
    sl = ctypes.c_int8(int(slot))
    s = np.ascontiguousarray(s3, dtype=np.float64).copy()
    lost = ctypes.c_int(0)
    ns = lib3().o3_move(ctypes.byref(sim.ms), ctypes.byref(t), ctypes.byref(sl), _p(s),
                        float(dr[0]), float(dr[1]), float(dr[2]), qdt, _p(cur), cap,
                        ctypes.byref(lost))
    return t.value, sl.value, s, bool(lost.value), ns, cur
