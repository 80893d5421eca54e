"""Seeded synthetic inputs: meshes, particle samplers and workload definitions.

This module produces the *inputs* that both the HIP library and the CPU
oracle consume: node coordinates, triangle connectivity, periodic image
shifts, particle positions in barycentric form and particle momenta.  It
holds none of the method's arithmetic (no Whitney forms, no pushers, no
tracking, no deposit, no field update); barycentric coordinates appear here
only as the coordinates in which a particle position is handed over.

Mesh recipe (shared by every workload):
  * nodes on a regular grid, interior nodes jittered uniformly by +-0.3 h,
    nodes on a non-periodic boundary slide only along that boundary and
    corners stay fixed;
  * periodic directions are triangulated by Delaunay of the point set plus
    its images within a margin of the period, keeping the triangles whose
    centroid lies in the central period cell; node ids are identified
    modulo the period and each triangle vertex records the image shift it
    was taken from, so every triangle is geometrically valid;
  * triangles are oriented counter-clockwise and numbered along a Morton
    curve of their centroids (locality of the per-triangle tables).

Particle positions are drawn as (triangle, barycentric pair): a triangle is
chosen with probability proportional to its area and the point uniformly
inside it.  The stored pair is (lambda_1, lambda_2) of the triangle's local
nodes 1 and 2 and the "derived slot" is local node 0, whose coordinate is
1 - lambda_1 - lambda_2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA-2018 constants (SI).
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
C_LIGHT = 299792458.0
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6

MESH_SEED = 1707
PARTICLE_SEED = 4333


@dataclasses.dataclass
class Mesh:
    node_xy: np.ndarray          # float64 [n_nodes, 2]
    tri_nodes: np.ndarray        # int32 [n_tris, 3], CCW
    tri_shift: np.ndarray | None  # int8 [n_tris, 3, 2] image shift per vertex, or None
    period: np.ndarray | None    # float64 [2]: period per axis (0 = not periodic), or None
    bbox: tuple                  # (x0, y0, x1, y1) of the domain

    @property
    def n_nodes(self):
        return int(self.node_xy.shape[0])

    @property
    def n_tris(self):
        return int(self.tri_nodes.shape[0])

    def vertex_xy(self) -> np.ndarray:
        """Image-consistent vertex coordinates, float64 [n_tris, 3, 2]."""
        v = self.node_xy[self.tri_nodes]
        if self.tri_shift is not None:
            v = v + self.tri_shift.astype(np.float64) * self.period[None, None, :]
        return v

    def tri_area(self) -> np.ndarray:
        v = self.vertex_xy()
        return 0.5 * ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
                      - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))

    def centroids(self) -> np.ndarray:
        return self.vertex_xy().mean(axis=1)


def _morton_order(xy: np.ndarray, bbox) -> np.ndarray:
    x0, y0, x1, y1 = bbox
    q = np.empty((xy.shape[0], 2), dtype=np.uint64)
    q[:, 0] = np.clip((xy[:, 0] - x0) / (x1 - x0) * 65535.0, 0, 65535).astype(np.uint64)
    q[:, 1] = np.clip((xy[:, 1] - y0) / (y1 - y0) * 65535.0, 0, 65535).astype(np.uint64)

    def spread(v):
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1))
    return np.argsort(code, kind="stable")


def grid_mesh(nx: int, ny: int, lx: float, ly: float, periodic_x: bool = False,
              periodic_y: bool = False, seed: int = MESH_SEED, jitter: float = 0.3,
              grade: float = 1.0) -> Mesh:
    """Jittered-grid Delaunay mesh of [0,lx] x [0,ly].

    nx, ny count grid nodes per axis; a periodic axis has its nodes on
    [0, l) with spacing l/n, a bounded axis on [0, l] with spacing l/(n-1).
    ``grade`` > 1 maps the grid through a smooth tensor-product stretching
    whose largest/smallest spacing ratio is ``grade`` (finest at the
    centre); it is only used with bounded axes.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    sx = np.arange(nx, dtype=np.float64) / (nx if periodic_x else nx - 1)
    sy = np.arange(ny, dtype=np.float64) / (ny if periodic_y else ny - 1)
    hx = 1.0 / (nx if periodic_x else nx - 1)
    hy = 1.0 / (ny if periodic_y else ny - 1)
    S, T = np.meshgrid(sx, sy, indexing="xy")
    S = S.reshape(-1)
    T = T.reshape(-1)
    js = rng.uniform(-jitter, jitter, S.shape) * hx
    jt = rng.uniform(-jitter, jitter, T.shape) * hy
    on_x_bnd = ((S == 0.0) | (S == 1.0)) & (not periodic_x)
    on_y_bnd = ((T == 0.0) | (T == 1.0)) & (not periodic_y)
    js[on_x_bnd] = 0.0
    jt[on_y_bnd] = 0.0
    S = S + js
    T = T + jt
    if periodic_x:
        S = np.mod(S, 1.0)
    if periodic_y:
        T = np.mod(T, 1.0)
    if grade != 1.0:
        if periodic_x or periodic_y:
            raise ValueError("graded meshes are bounded in both axes")
        S = _grade_map(S, grade)
        T = _grade_map(T, grade)
    pts = np.stack([S * lx, T * ly], axis=1)
    n = pts.shape[0]
    period = np.array([lx if periodic_x else 0.0, ly if periodic_y else 0.0])

    # Images within a margin of the period cell for the periodic axes.
    margin_x = 4.0 * hx * lx
    margin_y = 4.0 * hy * ly
    shifts_x = (-1, 0, 1) if periodic_x else (0,)
    shifts_y = (-1, 0, 1) if periodic_y else (0,)
    all_pts, all_ids, all_sh = [], [], []
    for dx in shifts_x:
        for dy in shifts_y:
            p = pts + np.array([dx * lx, dy * ly])
            keep = np.ones(n, dtype=bool)
            if dx != 0:
                keep &= (p[:, 0] > -margin_x) & (p[:, 0] < lx + margin_x)
            if dy != 0:
                keep &= (p[:, 1] > -margin_y) & (p[:, 1] < ly + margin_y)
            idx = np.nonzero(keep)[0]
            all_pts.append(p[idx])
            all_ids.append(idx)
            all_sh.append(np.tile(np.array([dx, dy], dtype=np.int8), (idx.size, 1)))
    P = np.concatenate(all_pts)
    ID = np.concatenate(all_ids)
    SH = np.concatenate(all_sh)
    dl = Delaunay(P)
    if len(dl.coplanar) != 0:
        raise RuntimeError("Delaunay dropped points")
    simp = dl.simplices
    cen = P[simp].mean(axis=1)
    keep = np.ones(simp.shape[0], dtype=bool)
    if periodic_x:
        keep &= (cen[:, 0] >= 0.0) & (cen[:, 0] < lx)
    if periodic_y:
        keep &= (cen[:, 1] >= 0.0) & (cen[:, 1] < ly)
    simp = simp[keep]
    tri = ID[simp].astype(np.int32)
    shift = SH[simp].astype(np.int8)
    v = P[simp]
    a2 = ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
          - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))
    flip = a2 < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    shift[flip] = shift[flip][:, [0, 2, 1]]
    a2 = np.abs(a2)
    # Drop zero-area slivers along straight boundaries (collinear hull points).
    good = a2 > 1e-12 * (lx * ly) / max(1, tri.shape[0])
    tri, shift, cen = tri[good], shift[good], cen[keep][good]
    order = _morton_order(cen, (0.0, 0.0, lx, ly))
    tri = np.ascontiguousarray(tri[order])
    shift = np.ascontiguousarray(shift[order])
    if not (periodic_x or periodic_y):
        shift = None
        period = None
    m = Mesh(node_xy=pts, tri_nodes=tri, tri_shift=shift, period=period,
             bbox=(0.0, 0.0, lx, ly))
    if np.any(m.tri_area() <= 0):
        raise RuntimeError("non-positive triangle area")
    return m


def _grade_map(s: np.ndarray, ratio: float) -> np.ndarray:
    """Monotone map of [0,1] onto itself whose slope at the ends is
    ``ratio`` times its slope at the centre (spacing ratio ``ratio``)."""
    # phi(s) = s + a * (s - 1/2)^3 style map with phi(0)=0, phi(1)=1:
    # phi'(s) = k (1 + b (2s-1)^2); ratio = 1 + b; k from phi(1) = 1.
    b = ratio - 1.0
    k = 1.0 / (1.0 + b / 3.0)
    x = 2.0 * s - 1.0
    return 0.5 * (1.0 + k * (x + b * x ** 3 / 3.0))


# ---------------------------------------------------------------------------
# Particle samplers
# ---------------------------------------------------------------------------

def sample_in_triangles(mesh: Mesh, n: int, rng, tri_mask=None):
    """Uniform positions: triangle with probability proportional to area,
    point uniform inside it.  Returns (tri int32, lam float64 [n,2]) with the
    stored pair (lambda_1, lambda_2) and local node 0 derived."""
    area = mesh.tri_area()
    w = area.copy()
    if tri_mask is not None:
        w = np.where(tri_mask, w, 0.0)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    tri = np.searchsorted(cdf, rng.random(n), side="right").astype(np.int32)
    tri = np.minimum(tri, mesh.n_tris - 1)
    r1 = np.sqrt(rng.random(n))
    r2 = rng.random(n)
    lam = np.empty((n, 2), dtype=np.float64)
    lam[:, 0] = r1 * (1.0 - r2)
    lam[:, 1] = r1 * r2
    return tri, lam


def bary_to_xy(mesh: Mesh, tri: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Cartesian position of (tri, stored pair) inputs (slot 0 derived)."""
    v = mesh.vertex_xy()[tri]
    l0 = 1.0 - lam[:, 0] - lam[:, 1]
    return l0[:, None] * v[:, 0] + lam[:, 0:1] * v[:, 1] + lam[:, 1:2] * v[:, 2]


def locate_points(mesh: Mesh, xy: np.ndarray):
    """Point location for input generation: for each point, the lowest-id
    triangle containing it and its barycentric pair (lambda_1, lambda_2).
    Uses a bucket grid over triangle bounding boxes."""
    v = mesh.vertex_xy()
    # bucket grid over the triangle frames (periodic frames extend past the cell)
    x0, y0 = v[:, :, 0].min(), v[:, :, 1].min()
    x1, y1 = v[:, :, 0].max(), v[:, :, 1].max()
    nb = max(1, int(math.sqrt(mesh.n_tris / 2)))
    bx = (x1 - x0) / nb
    by = (y1 - y0) / nb
    lo = np.floor((v.min(axis=1) - [x0, y0]) / [bx, by]).astype(np.int64)
    hi = np.floor((v.max(axis=1) - [x0, y0]) / [bx, by]).astype(np.int64)
    lo = np.clip(lo, 0, nb - 1)
    hi = np.clip(hi, 0, nb - 1)
    buckets = [[] for _ in range(nb * nb)]
    for t in range(mesh.n_tris):
        for i in range(lo[t, 0], hi[t, 0] + 1):
            for j in range(lo[t, 1], hi[t, 1] + 1):
                buckets[j * nb + i].append(t)
    out_t = np.full(xy.shape[0], -1, dtype=np.int32)
    out_l = np.zeros((xy.shape[0], 2))
    for p in range(xy.shape[0]):
        best = None
        for q in _images(mesh, xy[p]):
            qi = int(np.clip(np.floor((q[0] - x0) / bx), 0, nb - 1))
            qj = int(np.clip(np.floor((q[1] - y0) / by), 0, nb - 1))
            for t in sorted(buckets[qj * nb + qi]):
                if best is not None and t >= best[0]:
                    break
                a, b, c = v[t]
                den = (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1])
                l1 = ((q[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (q[1] - a[1])) / den
                l2 = ((b[0] - a[0]) * (q[1] - a[1]) - (q[0] - a[0]) * (b[1] - a[1])) / den
                if l1 >= 0 and l2 >= 0 and l1 + l2 <= 1:
                    best = (t, l1, l2)
                    break
        if best is None:
            raise ValueError(f"point {xy[p]} is outside the mesh")
        out_t[p] = best[0]
        out_l[p] = best[1:]
    return out_t, out_l


def _images(mesh: Mesh, q):
    """The point and its images one period away along periodic axes."""
    px, py = (0.0, 0.0) if mesh.period is None else (float(mesh.period[0]), float(mesh.period[1]))
    out = []
    for sx in ((-1, 0, 1) if px > 0 else (0,)):
        for sy in ((-1, 0, 1) if py > 0 else (0,)):
            out.append((q[0] + sx * px, q[1] + sy * py))
    return out


def sample_mj2d(n: int, theta: float, rng) -> np.ndarray:
    """Magnitude of the normalised momentum p/(m c) for an in-plane
    Maxwell-Juttner equilibrium f(p) d^2p ~ exp(-gamma/theta) d^2p.

    With p dp = gamma dgamma the density of x = gamma - 1 is proportional to
    (1 + x) exp(-x/theta): a mixture of Gamma(1, theta) (weight 1/(1+theta))
    and Gamma(2, theta) (weight theta/(1+theta)), sampled exactly."""
    pick = rng.random(n) < 1.0 / (1.0 + theta)
    x = np.where(pick, rng.gamma(1.0, theta, n), rng.gamma(2.0, theta, n))
    g = 1.0 + x
    return np.sqrt(g * g - 1.0)


@dataclasses.dataclass
class Species:
    name: str
    q: float        # charge of the physical particle [C]
    m: float        # rest mass [kg]
    w: float        # macro weight: physical particles per metre of depth
    tri: np.ndarray
    lam: np.ndarray  # [n, 2] stored pair, slot 0 derived
    u: np.ndarray    # [n, 2] u = gamma v [m/s]

    @property
    def n(self):
        return int(self.tri.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    species: list
    dt: float
    steps: int
    pusher: str
    precision: str
    bz_ext: float = 0.0                  # uniform external Bz [T]
    e_affine: np.ndarray | None = None   # [E0x, E0y, Kxx, Kxy, Kyx, Kyy]
    spai_level: int = 1
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_particles(self):
        return sum(s.n for s in self.species)


def cyclotron(seed_offset: int = 0, n_particles: int = 64, n_side: int = 33) -> Workload:
    """Relativistic cyclotron: 1 m square, PEC walls, uniform Bz = 1 T,
    electrons at random positions in [0.1, 0.9]^2 with gamma ~ U[1.5, 10]
    and in-plane momentum of random direction; dt = 0.2 m_e / (e B)."""
    mesh = grid_mesh(n_side, n_side, 1.0, 1.0)
    rng = np.random.default_rng(PARTICLE_SEED + 0 + seed_offset)
    cen = mesh.centroids()
    mask = (cen[:, 0] > 0.1) & (cen[:, 0] < 0.9) & (cen[:, 1] > 0.1) & (cen[:, 1] < 0.9)
    tri, lam = sample_in_triangles(mesh, n_particles, rng, mask)
    g = rng.uniform(1.5, 10.0, n_particles)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_particles)
    um = C_LIGHT * np.sqrt(g * g - 1.0)
    u = np.stack([um * np.cos(ang), um * np.sin(ang)], axis=1)
    B = 1.0
    dt = 0.2 * M_E / (E_CHARGE * B)
    sp = Species("electron", -E_CHARGE, M_E, 1.0, tri, lam, u)
    return Workload("cyclotron", mesh, [sp], dt, 5000, "boris", "fp64", bz_ext=B,
                    spai_level=2, extra={"gamma0": g})


def synchrocyclotron(case: str = "synched", n_side: int = 50, steps: int = 5000,
                     steps_per_period: int = 1000) -> Workload:
    """Synchrocyclotron of Sec. III.A: one electron injected at (0.52, 0.5) m
    with |v| = 1e7 m/s along +y on the PEC unit square; B_z = m v0/(e r0)
    (r0 = 0.02 m, 2.84281e-3 T) over the magnet region, a disk of radius
    0.45 m about the centre, and zero outside it; a vertical accelerating
    gap of width 0.02 m centred at x = 0.5 carries the RF field
    E_x = E0 sin(phase), E0 = 2e5 V/m, applied as edge DoFs whose amplitude
    the driver sets each step.  case: "nonrel" (gamma held at 1, constant
    frequency f0 = eB/(2 pi m)), "unsynched" (relativistic, f0) or "synched"
    (relativistic, f0/gamma).  dt = 1/(f0 steps_per_period)."""
    if case not in ("nonrel", "unsynched", "synched"):
        raise ValueError(case)
    mesh = grid_mesh(n_side, n_side, 1.0, 1.0)
    v0, r0, e0, gap = 1.0e7, 0.02, 2.0e5, 0.02
    B = M_E * v0 / (E_CHARGE * r0)
    f0 = E_CHARGE * B / (2.0 * math.pi * M_E)
    dt = 1.0 / (f0 * steps_per_period)
    cen = mesh.centroids()
    bz_tri = np.where(np.hypot(cen[:, 0] - 0.5, cen[:, 1] - 0.5) < 0.45, B, 0.0)
    xy = np.array([[0.5 + r0, 0.5]])
    tri, lam = locate_points(mesh, xy)
    gamma = 1.0 if case == "nonrel" else 1.0 / math.sqrt(1.0 - (v0 / C_LIGHT) ** 2)
    u = np.array([[0.0, gamma * v0]])
    sp = Species("electron", -E_CHARGE, M_E, 1.0, tri, lam, u)
    extra = {"bz_tri": bz_tri, "f0": f0, "e0": e0, "gap": gap, "gap_x": 0.5, "case": case,
             "B": B}
    if case == "nonrel":
        extra["c"] = 1.0e30   # particle kinematics without relativistic mass
    return Workload("synchrocyclotron_" + case, mesh, [sp], dt, steps, "boris_tan", "fp64",
                    spai_level=1, extra=extra)


def boosted_oscillator(n_particles: int = 1_000_000, n_side: int = 159,
                       amplitude: float = 1e-4) -> Workload:
    """Lorentz-boosted harmonic oscillation: 1 m square periodic in x, PEC
    in y; uniform Bz = 0.25 T and a static affine restoring field
    E_y = -k (y - 1/2) with k = c B / 0.4 m; positrons drift along x at
    gamma_b in {2, 5, 10} about the E x B equilibrium row and oscillate with
    a small transverse amplitude of random phase."""
    mesh = grid_mesh(n_side, n_side, 1.0, 1.0, periodic_x=True)
    rng = np.random.default_rng(PARTICLE_SEED + 1)
    B = 0.25
    k = C_LIGHT * B / 0.4
    yc = 0.5
    gb = np.array([2.0, 5.0, 10.0])[np.arange(n_particles) % 3]
    vd = C_LIGHT * np.sqrt(1.0 - 1.0 / gb ** 2)
    # Positron (q > 0): force q(E_y - v_d B) = 0 at the equilibrium row.
    yeq = yc - vd * B / k
    m, q = M_E, E_CHARGE
    w_lab = np.sqrt((q * k / m) / gb + (q * B / m) ** 2 / gb ** 4)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_particles)
    x = rng.uniform(0.0, 1.0, n_particles)
    y = yeq + amplitude * np.cos(phase)
    # Eigen-oscillation in the drift frame (non-relativistic there):
    # y' = A cos, u'_y = -A w' sin, u'_x = W' A cos with W' = qB/(gamma_b m)
    # (x-drift mode not excited); boosted back to the lab along x.
    w_drift = gb * w_lab
    big_w = q * B / (gb * m)
    upx = big_w * amplitude * np.cos(phase)
    upy = -amplitude * w_drift * np.sin(phase)
    gp = np.sqrt(1.0 + (upx ** 2 + upy ** 2) / C_LIGHT ** 2)
    ux = gb * (upx + vd * gp)
    uy = upy
    tri, lam = locate_points(mesh, np.stack([x, y], axis=1)) if n_particles <= 20000 else \
        _locate_fast(mesh, np.stack([x, y], axis=1))
    u = np.stack([ux, uy], axis=1)
    dt = 0.2 * m / (q * B)
    sp = Species("positron", q, m, 1.0, tri, lam, u)
    return Workload("boosted_oscillator", mesh, [sp], dt, 2000, "vay", "fp64", bz_ext=B,
                    e_affine=np.array([0.0, k * yc, 0.0, 0.0, 0.0, -k]),
                    extra={"gamma_b": gb, "omega_lab": w_lab, "k": k, "yc": yc})


def _locate_fast(mesh: Mesh, xy: np.ndarray):
    """Vectorised point location by a walk-free bucket search (input
    generation only; same result as ``locate_points`` for interior points)."""
    v = mesh.vertex_xy()
    # bucket grid over the triangle frames (periodic frames extend past the cell)
    x0, y0 = v[:, :, 0].min(), v[:, :, 1].min()
    x1, y1 = v[:, :, 0].max(), v[:, :, 1].max()
    nb = max(1, int(math.sqrt(mesh.n_tris / 2)))
    bx = (x1 - x0) / nb
    by = (y1 - y0) / nb
    lo = np.clip(np.floor((v.min(axis=1) - [x0, y0]) / [bx, by]).astype(np.int64), 0, nb - 1)
    hi = np.clip(np.floor((v.max(axis=1) - [x0, y0]) / [bx, by]).astype(np.int64), 0, nb - 1)
    # Candidate list per bucket as a CSR of (bucket, triangle) pairs.
    pairs_b, pairs_t = [], []
    for di in range(0, int((hi - lo)[:, 0].max()) + 1):
        for dj in range(0, int((hi - lo)[:, 1].max()) + 1):
            ok = (lo[:, 0] + di <= hi[:, 0]) & (lo[:, 1] + dj <= hi[:, 1])
            t = np.nonzero(ok)[0]
            pairs_b.append((lo[t, 1] + dj) * nb + lo[t, 0] + di)
            pairs_t.append(t)
    pb = np.concatenate(pairs_b)
    pt = np.concatenate(pairs_t)
    order = np.lexsort((pt, pb))
    pb, pt = pb[order], pt[order]
    start = np.searchsorted(pb, np.arange(nb * nb))
    end = np.searchsorted(pb, np.arange(nb * nb), side="right")
    out_t = np.full(xy.shape[0], np.iinfo(np.int32).max, dtype=np.int32)
    out_l = np.zeros((xy.shape[0], 2))
    maxc = int((end - start).max())
    px, py = (0.0, 0.0) if mesh.period is None else (float(mesh.period[0]), float(mesh.period[1]))
    for sx in ((-1, 0, 1) if px > 0 else (0,)):
        for sy in ((-1, 0, 1) if py > 0 else (0,)):
            q = xy + np.array([sx * px, sy * py])
            ok = (q[:, 0] >= x0) & (q[:, 0] <= x1) & (q[:, 1] >= y0) & (q[:, 1] <= y1)
            pi = np.clip(np.floor((q[:, 0] - x0) / bx).astype(np.int64), 0, nb - 1)
            pj = np.clip(np.floor((q[:, 1] - y0) / by).astype(np.int64), 0, nb - 1)
            bk = pj * nb + pi
            found = ~ok
            for c in range(maxc):
                todo = np.nonzero(~found)[0]
                if todo.size == 0:
                    break
                has = start[bk[todo]] + c < end[bk[todo]]
                found[todo[~has]] = True
                todo = todo[has]
                t = pt[start[bk[todo]] + c]
                a, b, cc = v[t, 0], v[t, 1], v[t, 2]
                p = q[todo]
                den = (b[:, 0] - a[:, 0]) * (cc[:, 1] - a[:, 1]) - (cc[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
                l1 = ((p[:, 0] - a[:, 0]) * (cc[:, 1] - a[:, 1]) - (cc[:, 0] - a[:, 0]) * (p[:, 1] - a[:, 1])) / den
                l2 = ((b[:, 0] - a[:, 0]) * (p[:, 1] - a[:, 1]) - (p[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])) / den
                inside = (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
                sel = todo[inside]
                found[sel] = True
                better = t[inside] < out_t[sel]
                out_t[sel[better]] = t[inside][better]
                out_l[sel[better], 0] = l1[inside][better]
                out_l[sel[better], 1] = l2[inside][better]
    if np.any(out_t == np.iinfo(np.int32).max):
        raise ValueError("points outside the mesh")
    return out_t, out_l


def pair_plasma(n_side: int = 316, length: float = 0.5, n_pairs: int = 8_000_000,
                theta: float = 0.1, B0: float = 1.0, seed_offset: int = 2,
                steps: int = 1000, precision: str = "mixed") -> Workload:
    """Relativistic pair-plasma Bernstein workload: doubly periodic square,
    electrons and positrons in collocated pairs with opposite momenta (zero
    initial charge and current), in-plane Maxwell-Juttner momenta of
    temperature theta = kT/(m c^2), uniform B0 with omega_c/omega_p = 2,
    dt = min(0.2/omega_c, 0.22 h/c)."""
    mesh = grid_mesh(n_side, n_side, length, length, periodic_x=True, periodic_y=True)
    rng = np.random.default_rng(PARTICLE_SEED + seed_offset)
    tri, lam = sample_in_triangles(mesh, n_pairs, rng)
    p = sample_mj2d(n_pairs, theta, rng)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_pairs)
    u = np.stack([C_LIGHT * p * np.cos(ang), C_LIGHT * p * np.sin(ang)], axis=1)
    wc = E_CHARGE * B0 / M_E
    wp = wc / 2.0
    n0 = wp * wp * EPS0 * M_E / (E_CHARGE * E_CHARGE)   # per species [m^-3]
    weight = n0 * length * length / n_pairs            # per metre of depth
    # 0.2/omega_c, capped by the leapfrog limit of the mesh (c dt/h <= 0.22;
    # the measured limit with SPAI(1) is about 0.27)
    dt = min(0.2 / wc, 0.22 * (length / n_side) / C_LIGHT)
    el = Species("electron", -E_CHARGE, M_E, weight, tri, lam, u)
    po = Species("positron", E_CHARGE, M_E, weight, tri.copy(), lam.copy(), -u)
    return Workload("pair_plasma_bernstein", mesh, [el, po], dt, steps, "boris", precision,
                    bz_ext=B0, spai_level=1,
                    extra={"omega_c": wc, "omega_p": wp, "n0": n0, "theta": theta})


def bernstein_strip(n_x: int = 428, n_y: int = 8, length_x: float = 0.0214,
                    theta: float = 0.005, ppc: int = 200, B0: float = 1.0, ratio: float = 2.0,
                    seed_offset: int = 5, precision: str = "mixed") -> Workload:
    """Pair plasma on a thin doubly periodic strip for the Bernstein
    dispersion of Sec. III.C (the paper's run is a long strip of width
    one gyroradius): n_x x n_y jittered cells of side length_x/n_x, ppc
    collocated pairs per triangle with opposite in-plane Maxwell-Juttner
    momenta of temperature theta, uniform B0, omega_c/omega_p = ratio per
    species, dt = min(0.2/omega_c, 0.22 h/c).  The default theta = 0.005
    (v_th = 0.07c) is the paper's non-relativistic example."""
    h = length_x / n_x
    length_y = n_y * h
    mesh = grid_mesh(n_x, n_y, length_x, length_y, periodic_x=True, periodic_y=True)
    n_pairs = ppc * mesh.n_tris
    rng = np.random.default_rng(PARTICLE_SEED + seed_offset)
    tri, lam = sample_in_triangles(mesh, n_pairs, rng)
    p = sample_mj2d(n_pairs, theta, rng)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_pairs)
    u = np.stack([C_LIGHT * p * np.cos(ang), C_LIGHT * p * np.sin(ang)], axis=1)
    wc = E_CHARGE * B0 / M_E
    wp = wc / ratio
    n0 = wp * wp * EPS0 * M_E / (E_CHARGE * E_CHARGE)
    weight = n0 * length_x * length_y / n_pairs
    dt = min(0.2 / wc, 0.22 * h / C_LIGHT)
    el = Species("electron", -E_CHARGE, M_E, weight, tri, lam, u)
    po = Species("positron", E_CHARGE, M_E, weight, tri.copy(), lam.copy(), -u)
    return Workload("bernstein_strip", mesh, [el, po], dt, 32768, "boris", precision,
                    bz_ext=B0, spai_level=1,
                    extra={"omega_c": wc, "omega_p": wp, "n0": n0, "theta": theta,
                           "length_x": length_x, "length_y": length_y})


def pair_plasma_small(**kw) -> Workload:
    """The 1/16-area copy of the pair-plasma workload (same density and
    temperature): 0.125 m square, 79 x 79 torus, 1M particles."""
    args = dict(n_side=79, length=0.125, n_pairs=500_000)
    args.update(kw)
    return pair_plasma(**args)


def batched_sweep(n_runs: int = 64, cell: float = 1.58e-3, seed: int = 10000,
                  tri_range=(2_000, 100_000), particle_range=(50_000, 4_000_000),
                  precision: str = "mixed") -> list:
    """Parameter sweep of independent pair-plasma runs with uneven sizes:
    run r (seed 10000 + r) draws its triangle count and particle count
    log-uniformly from the given ranges, B0 log-uniform in [0.5, 2] T and
    theta log-uniform in [0.05, 1]; omega_c/omega_p = 2 and dt = 0.2/omega_c
    per run; doubly periodic squares of cell size ``cell``."""
    out = []
    for r in range(n_runs):
        rng = np.random.default_rng(seed + r)
        nf = float(np.exp(rng.uniform(np.log(tri_range[0]), np.log(tri_range[1]))))
        npart = float(np.exp(rng.uniform(np.log(particle_range[0]), np.log(particle_range[1]))))
        B0 = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        theta = float(np.exp(rng.uniform(np.log(0.05), np.log(1.0))))
        n_side = max(4, int(round(np.sqrt(nf / 2.0))))
        w = pair_plasma(n_side=n_side, length=n_side * cell, n_pairs=max(1, int(npart) // 2),
                        theta=theta, B0=B0, seed_offset=seed + r - PARTICLE_SEED,
                        precision=precision)
        w.name = f"sweep_{r}"
        out.append(w)
    return out


def large_run(n_side: int = 708, n_particles: int = 128_000_000, grade: float = 10.0,
              layer: float = 0.1, beam_fraction: float = 0.05, beam_gamma: float = 20.0,
              theta: float = 0.5, B0: float = 1.0, precision: str = "mixed") -> Workload:
    """Large single run: graded jittered mesh of the unit square (spacing
    ratio ``grade``, finest at the centre) with PEC walls and an absorbing
    outer layer of width ``layer`` whose conductivity rises as (depth/w)^3;
    electrons with positions uniform by area, 95% in-plane Maxwell-Juttner
    at theta and 5% a beam of gamma 20 along +x; B0 uniform with
    omega_c/omega_p = 2; dt the smaller of 0.2/omega_c and 0.2 h_min/c.
    Immobile neutralising ions sit at the electrons' initial positions: with
    d^0 = 0 they are the initial charge q^0 of the Gauss accounting."""
    mesh = grid_mesh(n_side, n_side, 1.0, 1.0, grade=grade)
    rng = np.random.default_rng(PARTICLE_SEED + 4)
    tri, lam = sample_in_triangles(mesh, n_particles, rng)
    nb = int(round(beam_fraction * n_particles))
    p = sample_mj2d(n_particles - nb, theta, rng)
    ang = rng.uniform(0.0, 2.0 * math.pi, n_particles - nb)
    u = np.empty((n_particles, 2))
    u[:n_particles - nb, 0] = C_LIGHT * p * np.cos(ang)
    u[:n_particles - nb, 1] = C_LIGHT * p * np.sin(ang)
    u[n_particles - nb:, 0] = C_LIGHT * math.sqrt(beam_gamma ** 2 - 1.0)
    u[n_particles - nb:, 1] = 0.0
    wc = E_CHARGE * B0 / M_E
    wp = wc / 2.0
    n0 = wp * wp * EPS0 * M_E / (E_CHARGE * E_CHARGE)
    weight = n0 * 1.0 / n_particles
    area = mesh.tri_area()
    h_min = float(np.sqrt(2.0 * area.min()))
    dt = min(0.2 / wc, 0.2 * h_min / C_LIGHT)
    # absorbing layer conductivity per triangle, graded cubically with depth
    cen = mesh.centroids()
    depth = np.maximum(0.0, layer - np.minimum.reduce([cen[:, 0], 1.0 - cen[:, 0],
                                                      cen[:, 1], 1.0 - cen[:, 1]]))
    sigma_max = 0.5 * EPS0 / dt  # sigma dt / (2 eps0) reaches 1/4 at the wall
    sigma = sigma_max * (depth / layer) ** 3
    sp = Species("electron", -E_CHARGE, M_E, weight, tri, lam, u)
    return Workload("large_graded_absorbing", mesh, [sp], dt, 500, "hc", precision,
                    bz_ext=B0, spai_level=1,
                    extra={"omega_c": wc, "omega_p": wp, "sigma_tri": sigma, "theta": theta,
                           "h_min": h_min})


def wave_channel(nx: int = 161, ny: int = 6, length: float = 0.8, layer: float = 0.2,
                 sigma_dt: float = 0.1, pulse_width: float = 0.03, b_peak: float = 1e-3,
                 seed: int = MESH_SEED) -> Workload:
    """Field-only absorbing-layer workload: the channel [0, length] x [0, W),
    periodic in y (W = ny cells of the x spacing h = length/(nx - 1)), PEC
    at x = 0 and x = length, with absorbing layers of width ``layer`` at
    both ends whose conductivity rises as (depth/layer)^3 to sigma_max,
    sigma_max dt / eps0 = ``sigma_dt``; dt = 0.2 h/c.  Initial state: a
    Gaussian B_z pulse of peak ``b_peak`` [T] and 1/e half width
    ``pulse_width`` at the channel's centre (face fluxes b_f = B_z(centroid)
    A_f, d = 0), which splits into two halves running in -x and +x; after
    ``extra['steps_return']`` steps a wave reflected at either end would be
    back in the central region."""
    h = length / (nx - 1)
    width = ny * h
    mesh = grid_mesh(nx, ny, length, width, periodic_y=True, seed=seed)
    dt = 0.2 * h / C_LIGHT
    cen = mesh.centroids()
    depth = np.maximum(0.0, np.maximum(layer - cen[:, 0], cen[:, 0] - (length - layer)))
    sigma = (sigma_dt * EPS0 / dt) * (depth / layer) ** 3
    b0 = b_peak * np.exp(-((cen[:, 0] - 0.5 * length) / pulse_width) ** 2) * mesh.tri_area()
    # half-way to the wall, into the layer and back, plus a quarter of the centre
    travel = (0.5 * length - layer) + 2.0 * layer + 0.25 * (length - 2.0 * layer)
    steps = int(round(travel / (C_LIGHT * dt)))
    return Workload("wave_channel", mesh, [], dt, steps, "boris", "fp64", spai_level=1,
                    extra={"sigma_tri": sigma, "b0": b0, "layer": layer, "length": length,
                           "width": width, "steps_return": steps})
