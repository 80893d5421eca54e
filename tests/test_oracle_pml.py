"""Pins of the oracle's uniaxial PML (the absorbing boundary of Sec. III.C,
built here from the stretched-coordinate medium eps0 diag(1/s, s),
mu0 s, s = 1 + sigma/(j w eps0), along the layer's normal n).

* Uniform fields in a torus filled with the layer have closed forms: a
  uniform E along n keeps d and grows linearly, E(t) = E(0)(1 + sigma t /
  eps0) (the stretched medium's response to a static normal field; in the
  discrete update the growth per step is c/(1 + c/2), c = sigma dt/eps0);
  a uniform E along t decays as (1 - c) per step (a conductivity sigma).
  These fix the split of [*eps] into its n and t parts, the signs of the
  two auxiliary fluxes and their rates.
* Oblique waves: a pulse train at 60 degrees leaving a channel through PML
  layers, against the same pulse in a channel long enough that nothing
  comes back (the reflected field is the difference in the central
  region): reflected energy below 1e-4 of the incident, while the matched
  layer without the auxiliary terms reflects more than 1e-3 (its normal
  field sees a conductivity instead of the stretched response).
* Gauss's law holds at every free node, in the layer too (the update of d
  is the lossless one; the auxiliary fluxes enter only e).
"""
import math

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _uniform_e(T, ex, ey):
    """Line-integral DoFs of a uniform field on every edge (image-consistent
    coordinates of an adjacent triangle)."""
    e = np.zeros(T.ne)
    v = T.vxy.reshape(-1, 3, 2)
    for k in range(3):
        a, b = (k + 1) % 3, (k + 2) % 3
        dx = v[:, b, 0] - v[:, a, 0]
        dy = v[:, b, 1] - v[:, a, 1]
        e[T.tri_edge[:, k]] = T.tri_sign[:, k] * (ex * dx + ey * dy)
    return e


@pytest.mark.parametrize("axis", [0, 1])
def test_uniform_fields_in_a_stretched_torus(oracle_lib, axis):
    w = I.pair_plasma(n_side=8, length=0.01, n_pairs=1, theta=0.1, steps=1)
    osim = oracle_lib.OracleSim(w.mesh, w.dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=-1)
    T = osim.T
    cdt = 0.02
    sigma = np.full(T.nf, cdt * I.EPS0 / w.dt)
    for normal in (True, False):
        P = oracle_lib.pml_setup(T, sigma, w.dt, I.EPS0, axis=axis)
        assert P["rows"].size == int(T.edge_free.sum())
        osim.pml, osim.damp_b = P, np.ascontiguousarray(P["damp_b"])
        along_x = (axis == 0) == normal
        e0 = _uniform_e(T, 1.0 if along_x else 0.0, 0.0 if along_x else 1.0)
        from oracle import csr_matvec
        osim.e = e0.copy()
        osim.d = csr_matvec(*osim.Meps, e0)
        osim.b = np.zeros(T.nf)
        n = 40
        osim.step(n)
        if normal:
            want = 1.0 + n * cdt / (1.0 + 0.5 * cdt)
        else:
            want = (1.0 - cdt) ** n
        assert np.abs(osim.e - want * e0).max() <= 1e-11 * np.abs(e0).max(), (normal, want)
        assert np.abs(osim.b).max() <= 1e-12 * np.abs(e0).max() * w.dt


def _submesh(mesh, keep):
    tri = mesh.tri_nodes[keep]
    used = np.unique(tri)
    remap = -np.ones(mesh.node_xy.shape[0], np.int64)
    remap[used] = np.arange(used.size)
    return I.Mesh(node_xy=mesh.node_xy[used].copy(), tri_nodes=remap[tri].astype(np.int32),
                  tri_shift=None if mesh.tri_shift is None else mesh.tri_shift[keep].copy(),
                  period=mesh.period, bbox=mesh.bbox)


def _reflection(oracle_lib, theta_deg, mode):
    """Energy of the reflected B_z in the central region of a channel
    [0, 0.6] m x [0, 0.1) m (periodic in y, PEC at the ends, layers 0.15 m
    deep), relative to the incident pulse's."""
    h, ny, L, lay, ext = 0.0025, 40, 0.6, 0.15, 0.8
    W = ny * h
    dt = 0.2 * h / I.C_LIGHT
    meshB = I.grid_mesh(int(round((L + 2 * ext) / h)) + 1, ny, L + 2 * ext, W,
                        periodic_y=True, jitter=0.0)
    meshB.node_xy[:, 0] -= ext
    cxB = meshB.node_xy[meshB.tri_nodes][..., 0].mean(axis=1)
    keep = (cxB > 0.0) & (cxB < L)
    meshA = _submesh(meshB, keep)
    th = math.radians(theta_deg)
    ky = 2 * math.pi * 2 / W
    k = ky / math.sin(th)
    kx = k * math.cos(th)

    def pulse(T):
        v = T.vxy.reshape(-1, 3, 2)
        mids = 0.5 * (v + v[:, [1, 2, 0], :])
        bz = np.exp(-((mids[..., 0] - 0.5 * L) / 0.04) ** 2) * np.cos(kx * mids[..., 0] +
                                                                      ky * mids[..., 1])
        return bz.mean(axis=1) * T.area

    n = int(round((0.5 * L + lay + 0.1) / (I.C_LIGHT * math.cos(th) * dt)))
    ref = oracle_lib.OracleSim(meshB, dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=2)
    ref.b = pulse(ref.T)
    ref.step(n)
    sim = oracle_lib.OracleSim(meshA, dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=2)
    cx = sim.T.vxy.reshape(-1, 3, 2)[..., 0].mean(axis=1)
    depth = np.maximum(0.0, np.maximum(lay - cx, cx - (L - lay)))
    sigma = (0.1 * I.EPS0 / dt) * (depth / lay) ** 3
    if mode == "pml":
        P = oracle_lib.pml_setup(sim.T, sigma, dt, I.EPS0, axis=0)
        sim.pml, sim.damp_b = P, np.ascontiguousarray(P["damp_b"])
    else:
        damp, damp_b, _ = oracle_lib.absorber_damp(sim.T, sigma, dt, I.EPS0)
        sim.damp, sim.damp_b = np.ascontiguousarray(damp), np.ascontiguousarray(damp_b)
    b0 = pulse(sim.T)
    sim.b = b0.copy()
    sim.step(n)
    fa = np.nonzero((cx > lay) & (cx < L - lay))[0]
    fb = np.nonzero(keep)[0][fa]
    H = 1.0 / (I.MU0 * sim.T.area[fa])
    assert np.allclose(sim.T.area[fa], ref.T.area[fb])
    return float(np.sum((sim.b[fa] - ref.b[fb]) ** 2 * H)) / float(np.sum(b0[fa] ** 2 * H))


def test_oblique_reflection_pml_below_1e4(oracle_lib):
    r_pml = _reflection(oracle_lib, 60, "pml")
    r_matched = _reflection(oracle_lib, 60, "matched")
    assert r_pml < 1e-4, r_pml
    assert r_matched > 1e-3, r_matched


def test_gauss_law_through_the_layer(oracle_lib):
    """Electrons and positrons crossing into PML layers at both ends of a
    strip (periodic in y, PEC at the ends): Gauss's law at every free node,
    the layer's included, to 1e-12."""
    m = I.grid_mesh(40, 8, 0.04, 0.008, periodic_y=True, seed=9)
    rng = np.random.default_rng(12)
    n = 3000
    tri, lam = I.sample_in_triangles(m, n, rng)
    g_ = rng.uniform(1.5, 4.0, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    um = I.C_LIGHT * np.sqrt(g_ * g_ - 1)
    u = np.stack([um * np.cos(ang), um * np.sin(ang)], 1)
    dt = 0.15 * (0.04 / 39) / I.C_LIGHT
    sp = [(-I.E_CHARGE, I.M_E, 2e9, tri, lam, u), (I.E_CHARGE, I.M_E, 2e9, tri, lam, -u)]
    osim = oracle_lib.OracleSim(m, dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1, bz_ext=0.05)
    cx = osim.T.vxy.reshape(-1, 3, 2)[..., 0].mean(axis=1)
    lay = 0.01
    depth = np.maximum(0.0, np.maximum(lay - cx, cx - (0.04 - lay)))
    P = oracle_lib.pml_setup(osim.T, (0.2 * I.EPS0 / dt) * (depth / lay) ** 3, dt, I.EPS0)
    osim.pml, osim.damp_b = P, np.ascontiguousarray(P["damp_b"])
    q0, d0 = osim.charge(), osim.d.copy()
    osim.step(80, "vay")
    free = osim.T.node_free.astype(bool)
    res = osim.T.divergence(osim.d - d0) - (osim.charge() - q0)
    qmax = max(np.abs(q0).max(), np.abs(osim.charge()).max())
    assert np.abs(res[free]).max() <= 1e-12 * qmax
    assert np.abs(P["psi"]).max() > 0 and np.abs(P["phi"]).max() > 0  # the layer is active
