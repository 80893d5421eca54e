"""Pins of the oracle's 2-D field update (Sec. II.A: Faraday with the
incidence C, Ampere with C^T, [*mu^-1] = diag(1/(mu0 A_f)) and the inverse
Hodge) by the resonant frequencies of a PEC square cavity.

The TE_mn modes of the unit square with PEC walls have B_z = cos(m pi x)
cos(n pi y) and omega = c pi sqrt(m^2 + n^2) (textbook).  The oracle is
started from the face fluxes of that B_z with e = d = 0 and stepped with its
own field update; the mode's amplitude, measured as the [*mu^-1]-weighted
projection of b on the initial b, oscillates at the discrete frequency
omega_d.  The leapfrog's own time error is removed exactly through
omega_h = (2/dt) asin(omega_d dt/2) (a discrete eigenvalue omega_h^2 of the
spatial operator oscillates at cos(omega_d dt) = 1 - (omega_h dt)^2/2), so
omega_h/omega - 1 is the spatial error of the Whitney discretisation:

  * with the exact inverse of [*eps] it falls as h^2 (lowest-order edge
    elements), by a factor 4 per halving of h on structured meshes;
  * a wrong scale of [*mu^-1] or of [*eps], a dropped term or a wrong sign
    in C or C^T moves or destroys the resonance and fails these bounds;
  * on the jittered meshes the workloads use, the sparse approximate
    inverse on the first power of the graph of [*eps] (the pattern every
    2-D workload uses) stays within 1e-3 of the exact frequency.  (On a
    structured mesh, whose Delaunay diagonals all run one way, the same
    pattern is 3% off; the second power is exact to rounding there.)
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from paper_1707_04333_amd import inputs as I


def _te_mode_frequency(oracle_lib, n, level, cfl, jitter, m=1, k=1, periods=2.0):
    mesh = I.grid_mesh(n, n, 1.0, 1.0, jitter=jitter)
    h = 1.0 / (n - 1)
    dt = cfl * h / I.C_LIGHT
    osim = oracle_lib.OracleSim(mesh, dt, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=level)
    T = osim.T
    v = T.vxy.reshape(-1, 3, 2)
    # face flux of B_z: the three edge-midpoint rule (exact for quadratics)
    mids = 0.5 * (v + v[:, [1, 2, 0], :])
    bz = np.cos(m * np.pi * mids[..., 0]) * np.cos(k * np.pi * mids[..., 1])
    b0 = bz.mean(axis=1) * T.area
    osim.b = b0.copy()
    H = 1.0 / (I.MU0 * T.area)
    norm = float(np.sum(b0 * b0 * H))
    w_exact = I.C_LIGHT * np.pi * math.hypot(m, k)
    nsteps = int(round(periods * 2.0 * np.pi / w_exact / dt))
    amp = np.empty(nsteps + 1)
    amp[0] = 1.0
    for s in range(nsteps):
        osim.step(1)
        amp[s + 1] = float(np.sum(osim.b * b0 * H)) / norm
    t = np.arange(nsteps + 1) * dt

    def residual(w):
        X = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        c = np.linalg.lstsq(X, amp, rcond=None)[0]
        return float(np.sum((X @ c - amp) ** 2))

    grid = np.linspace(0.8 * w_exact, 1.2 * w_exact, 401)
    j = int(np.argmin([residual(w) for w in grid]))
    wd = minimize_scalar(residual, bracket=(grid[j - 1], grid[j], grid[j + 1]), tol=1e-12).x
    wh = 2.0 / dt * math.asin(wd * dt / 2.0)
    # the fit explains the signal: one mode, no growth
    X = np.stack([np.cos(wd * t), np.sin(wd * t), np.ones_like(t)], axis=1)
    c = np.linalg.lstsq(X, amp, rcond=None)[0]
    assert np.abs(X @ c - amp).max() < 0.02
    return wh / w_exact - 1.0


def test_te11_converges_at_second_order_with_exact_inverse(oracle_lib):
    errs = [_te_mode_frequency(oracle_lib, n, -1, 0.3, 0.0) for n in (9, 17, 33)]
    assert all(e > 0 for e in errs), errs
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs
    assert errs[2] < 5e-4, errs


def test_te21_converges_with_exact_inverse(oracle_lib):
    e17 = _te_mode_frequency(oracle_lib, 17, -1, 0.3, 0.0, m=2, k=1)
    e9 = _te_mode_frequency(oracle_lib, 9, -1, 0.3, 0.0, m=2, k=1)
    assert 3.0 < e9 / e17 < 4.6 and abs(e17) < 5e-3, (e9, e17)


@pytest.mark.parametrize("n,level", [(17, -1), (33, 1), (33, 2)])
def test_te11_on_jittered_mesh_within_1e3(oracle_lib, n, level):
    """Jittered meshes like the workloads': the exact inverse, and the
    approximate inverses on the first and second graph power."""
    err = _te_mode_frequency(oracle_lib, n, level, 0.15, 0.3)
    assert abs(err) < 1e-3, err
