"""Whole-run pins of the oracle against closed forms of charged-particle
motion in uniform and boosted fields (Sec. III.A-B).

Cyclotron (uniform Bz, E = 0, negligible self-field): every pusher maps
u^{n-1/2} to a rotation of it by a fixed angle theta, so the positions are
the vertices of a regular polygon inscribed in a circle of radius
R = dt |u| / (2 gamma sin(theta/2)), period 2 pi dt / theta.  The continuum
values r = gamma m |v| / (|q| B), omega = |q| B / (gamma m) are approached
as omega dt -> 0: the relative gap is (omega dt)^2 / 8 for the Boris
radius, below 1e-4 for the fast (gamma >= 7.5) particles of the workload.

Lorentz-boosted oscillator (Sec. III.B): a positron drifting at gamma_b in
the E x B row of a linear restoring field E_y = -k (y - y_c) with uniform
Bz oscillates in the drift frame with omega'^2 = q k gamma_b / m +
(q B / (gamma_b m))^2 (B' = B / gamma_b, E' gradient gamma_b k), seen in the
lab at omega_lab = omega' / gamma_b.  Vay and Higuera-Cary reproduce it;
Boris does not capture the relativistic E x B drift."""
import math

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _circle_fit(xy):
    x, y = xy[:, 0], xy[:, 1]
    A = np.stack([x, y, np.ones_like(x)], 1)
    b = x * x + y * y
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    cx, cy = sol[0] / 2, sol[1] / 2
    R = math.sqrt(sol[2] + cx * cx + cy * cy)
    return cx, cy, R


def _hc_half_tan(u, bm):
    u2 = u * u / I.C_LIGHT ** 2
    bb = bm * bm
    G = 0.5 * ((1 + u2 - bb) + math.sqrt((1 + u2 - bb) ** 2 + 4 * bb))
    return bm / math.sqrt(G)


@pytest.mark.parametrize("pusher", ["boris", "boris_tan", "vay", "hc"])
def test_cyclotron_orbits(oracle_lib, pusher):
    w = I.cyclotron()
    sp = w.species[0]
    sim = oracle_lib.OracleSim(w.mesh, w.dt, [(sp.q, sp.m, sp.w, sp.tri, sp.lam, sp.u)],
                               I.EPS0, I.MU0, I.C_LIGHT, spai_level=w.spai_level,
                               bz_ext=w.bz_ext)
    n_steps = 2000
    traj = np.empty((n_steps + 1, sp.n, 2))
    traj[0] = sim.positions(sim.species[0])
    for i in range(n_steps):
        sim.step(1, pusher)
        traj[i + 1] = sim.positions(sim.species[0])
    assert sim.lost == 0
    um = np.linalg.norm(sp.u, axis=1)
    gam = np.sqrt(1 + um ** 2 / I.C_LIGHT ** 2)
    alpha = abs(sp.q) * w.dt / (2 * sp.m)
    bm = alpha * w.bz_ext
    worst_disc = 0.0
    worst_cont_fast = 0.0
    for p in range(sp.n):
        cx, cy, R = _circle_fit(traj[:, p])
        ang = np.unwrap(np.arctan2(traj[:, p, 1] - cy, traj[:, p, 0] - cx))
        theta = (ang[-1] - ang[0]) / n_steps
        assert theta > 0  # electrons gyrate counter-clockwise in +Bz
        g = gam[p]
        if pusher in ("boris", "vay"):
            th_ref = 2 * math.atan(bm / g)
        elif pusher == "boris_tan":
            th_ref = 2 * bm / g
        else:
            th_ref = 2 * math.atan(_hc_half_tan(um[p], bm))
        R_ref = w.dt * um[p] / (2 * g * math.sin(th_ref / 2))
        worst_disc = max(worst_disc, abs(R / R_ref - 1), abs(theta / th_ref - 1))
        r_cont = sp.m * um[p] / (abs(sp.q) * w.bz_ext)
        om_cont = abs(sp.q) * w.bz_ext / (g * sp.m)
        if g >= 7.5:
            worst_cont_fast = max(worst_cont_fast, abs(R / r_cont - 1),
                                  abs(theta / w.dt / om_cont - 1))
        if pusher == "boris_tan":
            # the tan correction makes the gyrofrequency exact at every gamma
            assert abs(theta / w.dt / om_cont - 1) < 1e-9
    assert worst_disc < 1e-9
    assert worst_cont_fast < 1e-4


def _fit_freq(t, y, w0):
    """Frequency of the best least-squares fit a cos wt + b sin wt + c:
    a scan over +-10% of w0 refined by golden-section search."""
    def rss(om):
        A = np.stack([np.cos(om * t), np.sin(om * t), np.ones_like(t)], 1)
        sol = np.linalg.lstsq(A, y, rcond=None)[0]
        return float(np.sum((A @ sol - y) ** 2))
    grid = w0 * np.linspace(0.9, 1.1, 801)
    i = int(np.argmin([rss(o) for o in grid]))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    for _ in range(60):
        m1, m2 = lo + (hi - lo) * 0.382, lo + (hi - lo) * 0.618
        if rss(m1) < rss(m2):
            hi = m2
        else:
            lo = m1
    return 0.5 * (lo + hi)


def test_boosted_oscillator(oracle_lib):
    w = I.boosted_oscillator(n_particles=6)
    sp = w.species[0]
    errs = {}
    for pusher in ("vay", "hc", "boris"):
        sim = oracle_lib.OracleSim(w.mesh, w.dt, [(sp.q, sp.m, sp.w, sp.tri, sp.lam, sp.u)],
                                   I.EPS0, I.MU0, I.C_LIGHT, spai_level=1, bz_ext=w.bz_ext,
                                   affine=w.e_affine)
        n_steps = 2000
        ys = np.empty((n_steps + 1, sp.n))
        ys[0] = sim.positions(sim.species[0])[:, 1]
        for i in range(n_steps):
            sim.step(1, pusher)
            ys[i + 1] = sim.positions(sim.species[0])[:, 1]
        assert sim.lost == 0
        t = np.arange(n_steps + 1) * w.dt
        e = []
        for p in range(sp.n):
            om = _fit_freq(t, ys[:, p], w.extra["omega_lab"][p])
            e.append(abs(om / w.extra["omega_lab"][p] - 1))
        errs[pusher] = max(e)
    # leapfrog error (w dt)^2/24 ~ 1.2e-4 at gamma_b = 2 plus the finite
    # amplitude term (gamma_b w A / c)^2 ~ 6e-5
    assert errs["vay"] < 5e-4 and errs["hc"] < 5e-4, errs
    assert errs["boris"] > 5 * max(errs["vay"], errs["hc"]), errs
