"""Seeded synthetic inputs for the tetrahedral (3-D) path: box meshes,
particle samplers and workload definitions.

Like ``inputs`` it holds none of the method's arithmetic; barycentric
coordinates appear only as the form in which a particle position is handed
over.

Mesh recipe:
  * nodes on a regular grid of the box, interior nodes jittered uniformly
    by +-jitter*h/2 per axis; nodes on a non-periodic face of the box slide
    only within that face;
  * every grid cell is split into the six tetrahedra that share its main
    diagonal (Kuhn's subdivision: from corner (0,0,0) to (1,1,1) one axis
    at a time, one tetrahedron per order of the axes), which is conforming
    across cells;
  * periodic axes identify nodes modulo the period and each tetrahedron
    vertex records the image shift it was taken from;
  * tetrahedra are positively oriented (det[x1-x0, x2-x0, x3-x0] > 0) and
    numbered along a Morton curve of their centroids.

Particle positions are drawn as (tetrahedron, barycentric triple): a
tetrahedron is chosen with probability proportional to its volume and the
point uniformly inside it.  The stored triple is (lambda_1, lambda_2,
lambda_3) of local nodes 1-3 and the derived slot is local node 0.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

from .inputs import C_LIGHT, E_CHARGE, EPS0, M_E, MESH_SEED, PARTICLE_SEED, Species, Workload


@dataclasses.dataclass
class TetMesh:
    node_xyz: np.ndarray          # float64 [n_nodes, 3]
    tet_nodes: np.ndarray         # int32 [n_tets, 4], positively oriented
    tet_shift: np.ndarray | None  # int8 [n_tets, 4, 3] image shift per vertex, or None
    period: np.ndarray | None     # float64 [3], 0 = not periodic, or None
    bbox: tuple                   # (x0, y0, z0, x1, y1, z1)

    @property
    def n_nodes(self):
        return int(self.node_xyz.shape[0])

    @property
    def n_tets(self):
        return int(self.tet_nodes.shape[0])

    def vertex_xyz(self) -> np.ndarray:
        v = self.node_xyz[self.tet_nodes]
        if self.tet_shift is not None:
            v = v + self.tet_shift.astype(np.float64) * self.period[None, None, :]
        return v

    def tet_volume(self) -> np.ndarray:
        v = self.vertex_xyz()
        a, b, c = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]
        return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0

    def centroids(self) -> np.ndarray:
        return self.vertex_xyz().mean(axis=1)


def _morton3(p: np.ndarray, lo, hi) -> np.ndarray:
    q = np.clip((p - lo) / (hi - lo) * 1023.0, 0, 1023).astype(np.uint64)

    def spread(v):
        v = (v | (v << np.uint64(16))) & np.uint64(0x030000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x0300F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x030C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x09249249)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def box_mesh(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
             periodic=(False, False, False), jitter: float = 0.2,
             seed: int = MESH_SEED) -> TetMesh:
    """Jittered Kuhn tetrahedral mesh of [0,lx] x [0,ly] x [0,lz].

    n* count grid nodes per axis; a periodic axis has its nodes on [0, l)
    with spacing l/n, a bounded axis on [0, l] with spacing l/(n-1)."""
    n = np.array([nx, ny, nz])
    L = np.array([lx, ly, lz], dtype=np.float64)
    per = np.array(periodic, dtype=bool)
    h = np.where(per, L / n, L / np.maximum(n - 1, 1))
    cells = np.where(per, n, n - 1)
    if np.any(cells < 1) or np.any(per & (n < 3)):
        raise ValueError("mesh too small")
    rng = np.random.default_rng(seed)
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    idx = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1)
    # node id = i + nx (j + ny k)
    order = idx[:, 0] + nx * (idx[:, 1] + ny * idx[:, 2])
    ijk = np.empty_like(idx)
    ijk[order] = idx
    xyz = ijk * h[None, :]
    disp = rng.uniform(-0.5, 0.5, size=xyz.shape) * jitter * h[None, :]
    for ax in range(3):
        if not per[ax]:
            on_face = (ijk[:, ax] == 0) | (ijk[:, ax] == n[ax] - 1)
            disp[on_face, ax] = 0.0
    xyz = xyz + disp
    c = np.stack(np.meshgrid(np.arange(cells[0]), np.arange(cells[1]), np.arange(cells[2]),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    tets, shifts = [], []
    for perm in itertools.permutations(range(3)):
        corner = np.zeros(3, dtype=np.int64)
        path = [corner.copy()]
        for ax in perm:
            corner[ax] += 1
            path.append(corner.copy())
        verts = np.stack([c + p[None, :] for p in path], axis=1)  # [ncell, 4, 3]
        sh = np.where(per[None, None, :], verts // n[None, None, :], 0)
        w = np.where(per[None, None, :], verts % n[None, None, :], verts)
        ids = w[..., 0] + nx * (w[..., 1] + ny * w[..., 2])
        tets.append(ids)
        shifts.append(sh)
    tet = np.concatenate(tets).astype(np.int32)
    shift = np.concatenate(shifts).astype(np.int8)
    period = np.where(per, L, 0.0)
    v = xyz[tet] + shift.astype(np.float64) * period[None, None, :]
    det = np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    neg = det < 0
    tet[neg, 2], tet[neg, 3] = tet[neg, 3].copy(), tet[neg, 2].copy()
    s2 = shift[neg, 2].copy()
    shift[neg, 2] = shift[neg, 3]
    shift[neg, 3] = s2
    m = TetMesh(xyz, tet, shift if per.any() else None, period if per.any() else None,
                (0.0, 0.0, 0.0, lx, ly, lz))
    if np.any(m.tet_volume() <= 0):
        raise ValueError("inverted tetrahedron: lower the jitter")
    o = _morton3(m.centroids(), np.zeros(3), L)
    m.tet_nodes = np.ascontiguousarray(m.tet_nodes[o])
    if m.tet_shift is not None:
        m.tet_shift = np.ascontiguousarray(m.tet_shift[o])
    return m


def sample_in_tets(mesh: TetMesh, n: int, rng, tet_mask=None):
    """Uniform positions: tetrahedron with probability proportional to its
    volume, point uniform inside it (barycentrics Dirichlet(1,1,1,1) from
    normalised exponentials).  Returns (tet int32, lam float64 [n,3]) with
    the stored triple (lambda_1, lambda_2, lambda_3), local node 0 derived."""
    w = mesh.tet_volume()
    if tet_mask is not None:
        w = np.where(tet_mask, w, 0.0)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    tet = np.minimum(np.searchsorted(cdf, rng.random(n), side="right"), mesh.n_tets - 1)
    x = rng.exponential(size=(n, 4))
    x /= x.sum(axis=1, keepdims=True)
    return tet.astype(np.int32), np.ascontiguousarray(x[:, 1:])


def bary_to_xyz(mesh: TetMesh, tet: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Cartesian position of (tet, stored triple) inputs (slot 0 derived)."""
    v = mesh.vertex_xyz()[tet]
    l0 = 1.0 - lam.sum(axis=1)
    return l0[:, None] * v[:, 0] + np.einsum("nk,nkd->nd", lam, v[:, 1:])


def sample_mj3d(n: int, theta: float, rng) -> np.ndarray:
    """Magnitude of p/(m c) for the 3-D Maxwell-Juttner equilibrium
    f(p) d^3p ~ exp(-gamma/theta) d^3p, exactly, by rejection from a Gamma
    mixture.  With x = gamma - 1 the density of x is proportional to
    (1 + x) sqrt(x (2 + x)) exp(-x/theta), which is at most
    sqrt(2) (x^1/2 + 2 x^3/2 + x^5/2) exp(-x/theta): a mixture of
    Gamma(3/2, theta), Gamma(5/2, theta) and Gamma(7/2, theta) with weights
    G(3/2) theta^3/2, 2 G(5/2) theta^5/2 and G(7/2) theta^7/2.  A draw x of
    the mixture is kept with probability sqrt(1 + x/2) / (1 + x), the ratio
    of the two (about 0.9 at theta = 0.1); then |u| = sqrt(x (2 + x))."""
    from math import gamma as G
    wts = np.array([G(1.5) * theta ** 1.5, 2.0 * G(2.5) * theta ** 2.5, G(3.5) * theta ** 3.5])
    wts /= wts.sum()
    parts, got, acc = [], 0, 0.5
    while got < n:
        m = int((n - got) / acc * 1.1) + 64
        shape = 1.5 + rng.choice(3, size=m, p=wts)
        x = rng.gamma(shape, theta)
        keep = rng.random(m) * (1.0 + x) < np.sqrt(1.0 + 0.5 * x)
        acc = max(float(keep.mean()), 0.01)
        parts.append(x[keep])
        got += parts[-1].size
    x = np.concatenate(parts)[:n]
    return np.sqrt(x * (2.0 + x))


def isotropic_directions(n: int, rng) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def tet_cyclotron(n_side: int = 7, n_particles: int = 32, seed_offset: int = 20,
                  b_dir=(0.36, 0.48, 0.8), B0: float = 1.0) -> Workload:
    """Relativistic gyration in 3-D: unit cube, PEC walls, uniform B of
    magnitude B0 along b_dir (not a mesh axis), electrons at random points
    of [0.3, 0.7]^3 with gamma ~ U[1.5, 4] and isotropic momentum
    directions (helical orbits); dt = 0.2 m_e / (e B0)."""
    mesh = box_mesh(n_side, n_side, n_side, 1.0, 1.0, 1.0)
    rng = np.random.default_rng(PARTICLE_SEED + seed_offset)
    cen = mesh.centroids()
    inner = np.all((cen > 0.3) & (cen < 0.7), axis=1)
    tet, lam = sample_in_tets(mesh, n_particles, rng, tet_mask=inner)
    g = rng.uniform(1.5, 4.0, n_particles)
    u = C_LIGHT * np.sqrt(g * g - 1.0)[:, None] * isotropic_directions(n_particles, rng)
    b = np.asarray(b_dir, dtype=np.float64)
    b = B0 * b / np.linalg.norm(b)
    dt = 0.2 * M_E / (E_CHARGE * B0)
    sp = Species("electron", -E_CHARGE, M_E, 1.0, tet, lam, u)
    return Workload("tet_cyclotron", mesh, [sp], dt, 400, "boris", "fp64", spai_level=1,
                    extra={"b_ext": b})


def tet_pair_plasma(n_side: int = 48, length: float = 0.048, n_pairs: int = 8_000_000,
                    theta: float = 0.1, B0: float = 1.0, seed_offset: int = 21,
                    steps: int = 200, courant: float = 0.12) -> Workload:
    """3-D pair plasma on a triply periodic cube: electrons and positrons
    in collocated pairs with opposite momenta (zero initial charge and
    current), isotropic 3-D Maxwell-Juttner momenta at temperature theta,
    uniform B0 along z with omega_c/omega_p = 2 per species,
    dt = min(0.2/omega_c, courant h/c)."""
    mesh = box_mesh(n_side, n_side, n_side, length, length, length, periodic=(True, True, True))
    rng = np.random.default_rng(PARTICLE_SEED + seed_offset)
    tet, lam = sample_in_tets(mesh, n_pairs, rng)
    p = sample_mj3d(n_pairs, theta, rng)
    u = C_LIGHT * p[:, None] * isotropic_directions(n_pairs, rng)
    wc = E_CHARGE * B0 / M_E
    wp = wc / 2.0
    n0 = wp * wp * EPS0 * M_E / (E_CHARGE * E_CHARGE)
    weight = n0 * length ** 3 / n_pairs
    dt = min(0.2 / wc, courant * (length / n_side) / C_LIGHT)
    el = Species("electron", -E_CHARGE, M_E, weight, tet, lam, u)
    po = Species("positron", E_CHARGE, M_E, weight, tet.copy(), lam.copy(), -u)
    return Workload("tet_pair_plasma", mesh, [el, po], dt, steps, "boris", "fp64",
                    spai_level=1,
                    extra={"b_ext": np.array([0.0, 0.0, B0]), "omega_c": wc, "omega_p": wp,
                           "n0": n0, "theta": theta})
