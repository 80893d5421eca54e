"""Pins of the absorbing layer (the stand-in for the PML of Sec. III.C).

  * a uniform magnetic field in a uniformly lossy torus decays as
    exp(-sigma t / eps0), the decay that a magnetic conductivity
    sigma_m = sigma mu0 / eps0 gives (dB/dt = -(sigma_m/mu0) B); the
    discrete factor per step agrees with it to O((sigma dt / eps0)^3) per
    step, and d stays at zero (a uniform field has no curl);
  * a pulse leaving a lossless channel through matched layers (electric and
    magnetic loss in that ratio) comes back with a reflected energy below
    1e-3 of what it carried, while the same layer with the electric loss
    alone reflects more than 5% (its wave impedance differs from free
    space);
  * without any layer the PEC walls send the whole pulse back (the
    measurement itself is sound)."""
import math

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _centre_energy(osim, w):
    """Field energy of the central, lossless part of the channel."""
    T = osim.T
    ptr, col, val = osim.Meps
    from oracle import csr_matvec
    Me_e = csr_matvec(ptr, col, val, osim.e)
    L, lay = w.extra["length"], w.extra["layer"]
    xy = w.mesh.node_xy
    mid = 0.5 * (xy[T.edge_lo, 0] + xy[T.edge_hi, 0])
    ce = (mid > lay) & (mid < L - lay)
    cx = w.mesh.centroids()[:, 0]
    cf = (cx > lay) & (cx < L - lay)
    WE = 0.5 * float(osim.e[ce] @ Me_e[ce])
    WB = 0.5 * float(np.sum(osim.b[cf] ** 2 / (osim.mu0 * T.area[cf])))
    return WE + WB


def _channel_run(oracle_lib, w, electric, magnetic, steps=None):
    osim = oracle_lib.OracleSim(w.mesh, w.dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=1)
    damp, damp_b, _ = oracle_lib.absorber_damp(osim.T, w.extra["sigma_tri"], w.dt, I.EPS0)
    if electric:
        osim.damp = np.ascontiguousarray(damp)
    if magnetic:
        osim.damp_b = np.ascontiguousarray(damp_b)
    osim.b = np.ascontiguousarray(w.extra["b0"], dtype=np.float64).copy()
    E0 = sum(osim.energies()[:2])
    osim.step(w.extra["steps_return"] if steps is None else steps)
    return osim, E0


def test_uniform_field_decays_at_matched_rate(oracle_lib):
    w = I.pair_plasma(n_side=8, length=0.01, n_pairs=1, theta=0.1, steps=1)
    B, sdt = 0.3, 0.02  # sigma dt / eps0
    osim = oracle_lib.OracleSim(w.mesh, w.dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=1)
    sigma = np.full(w.mesh.n_tris, sdt * I.EPS0 / w.dt)
    damp, damp_b, keep = oracle_lib.absorber_damp(osim.T, sigma, w.dt, I.EPS0)
    assert not keep.any()  # every node touches a lossy edge
    osim.damp, osim.damp_b = np.ascontiguousarray(damp), np.ascontiguousarray(damp_b)
    osim.b = B * osim.T.area
    n = 150
    osim.step(n)
    got = osim.b / (B * osim.T.area)
    cont = math.exp(-sdt * n)
    assert np.abs(got - got.mean()).max() <= 1e-13
    assert abs(got.mean() - cont) <= n * sdt ** 3 / 12.0 * cont * 1.01
    assert abs(got.mean() - cont) >= n * sdt ** 3 / 12.0 * cont * 0.9  # the O(x^3) term is there
    assert np.abs(osim.d).max() <= 1e-12 * B / I.MU0 * w.dt


def test_matched_layer_absorbs_pulse(oracle_lib):
    w = I.wave_channel()
    _, E0 = _channel_run(oracle_lib, w, False, False, steps=0)
    bare, _ = _channel_run(oracle_lib, w, False, False)
    el, _ = _channel_run(oracle_lib, w, True, False)
    matched, _ = _channel_run(oracle_lib, w, True, True)
    r_bare = _centre_energy(bare, w) / E0
    r_el = _centre_energy(el, w) / E0
    r_m = _centre_energy(matched, w) / E0
    assert r_bare > 0.8
    assert r_el > 0.05
    assert r_m < 1e-3
    # the energy left anywhere is small too: the layer took it up
    assert sum(matched.energies()[:2]) / E0 < 2e-3
