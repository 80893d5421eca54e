"""Pins of the oracle's scatter (Sec. II.D) and of discrete charge
conservation over whole runs (Sec. II.A eq. semi.dis.div.2, Sec. II.D eq.
full.dis.cont).

  * eq. I.assign is the exact line integral of W1 along a straight piece:
    its integrand is linear in the path parameter, so the midpoint rule
    evaluated from the Whitney basis itself is exact;
  * dipole identity: sum_e i_e t_e = Q dr / dt for a whole move, because
    sum_e t_e (W1_e . v) = v (W1 reproduces constants);
  * continuity node by node: q^{n+1} - q^n + dt S~ i^{n+1/2} = 0;
  * Gauss's law for the d = [*eps] e state: S~ (d^n - d^0) = q^n - q^0 over
    the whole run, at every free node, to rounding (the paper's tables
    report normalised residuals up to 5.2e-13)."""
import math

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _sim(oracle_lib, m, species=(), **kw):
    return oracle_lib.OracleSim(m, kw.pop("dt", 1e-12), list(species), I.EPS0, I.MU0,
                                I.C_LIGHT, **kw)


def test_segment_current_is_exact_line_integral(oracle_lib):
    m = I.grid_mesh(7, 7, 1.0, 1.0, seed=3)
    sim = _sim(oracle_lib, m)
    T = sim.T
    G = T.grad.reshape(-1, 3, 2)
    v = T.vxy.reshape(-1, 3, 2)
    rng = np.random.default_rng(1)
    f = int(np.nonzero(np.all(T.tri_nbr >= 0, axis=1))[0][0])
    for _ in range(50):
        Ls = rng.dirichlet([1, 1, 1])
        Lf = rng.dirichlet([1, 1, 1])
        xs, xf = Ls @ v[f], Lf @ v[f]
        dx = xf - xs
        pair = np.array([Ls[1], Ls[2]])
        ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, f, 0, pair, dx[0], dx[1],
                                                          qdt=1.0)
        assert ft == f and len(segs) == 1
        Lm = 0.5 * (Ls + Lf)
        for k in range(3):
            a, b = (k + 1) % 3, (k + 2) % 3
            W = Lm[a] * G[f, b] - Lm[b] * G[f, a]
            ref = T.tri_sign[f, k] * (W @ dx)
            assert abs(cur[T.tri_edge[f, k]] - ref) <= 1e-14


def test_dipole_identity_and_split_invariance(oracle_lib):
    m = I.grid_mesh(9, 9, 1.0, 1.0, seed=4)
    sim = _sim(oracle_lib, m)
    T = sim.T
    v = T.vxy.reshape(-1, 3, 2)
    # edge tangent lo -> hi
    tvec = np.zeros((T.ne, 2))
    for f in range(T.nf):
        for k in range(3):
            a, b = (k + 1) % 3, (k + 2) % 3
            tvec[T.tri_edge[f, k]] = T.tri_sign[f, k] * (v[f, b] - v[f, a])
    rng = np.random.default_rng(2)
    cen = v.mean(axis=1)
    inner = np.nonzero((cen[:, 0] > 0.3) & (cen[:, 0] < 0.7) & (cen[:, 1] > 0.3) & (cen[:, 1] < 0.7))[0]
    for _ in range(40):
        f = int(rng.choice(inner))
        pair = rng.dirichlet([1, 1, 1])[1:]
        ang = rng.uniform(0, 2 * np.pi)
        d = rng.uniform(0.01, 0.25) * np.array([np.cos(ang), np.sin(ang)])
        _, _, _, lost, segs, cur = oracle_lib.move_one(sim, f, 0, pair, d[0], d[1], qdt=1.0)
        assert not lost
        dip = cur @ tvec
        assert np.abs(dip - d).max() <= 1e-14 * 10
        # two half moves deposit the same total current
        t1, s1, p1, _, _, c1 = oracle_lib.move_one(sim, f, 0, pair, d[0] / 2, d[1] / 2)
        _, _, _, _, _, c2 = oracle_lib.move_one(sim, t1, s1, p1, d[0] / 2, d[1] / 2)
        assert np.abs(c1 + c2 - cur).max() <= 1e-14


def _charge_and_div(sim):
    return sim.charge(), sim.T.divergence(sim.d)


@pytest.mark.parametrize("pusher", ["boris", "vay", "hc", "boris_tan"])
def test_continuity_every_step_with_wall_losses(oracle_lib, pusher):
    """Fast electrons in a small PEC box with a weak B: many cross edges and
    many are lost at the walls; continuity holds at every free node and
    every step, and Gauss's law over the whole run."""
    m = I.grid_mesh(12, 12, 0.1, 0.1, seed=8)
    rng = np.random.default_rng(5)
    n = 3000
    tri, lam = I.sample_in_triangles(m, n, rng)
    g = rng.uniform(1.2, 4.0, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    um = I.C_LIGHT * np.sqrt(g * g - 1)
    u = np.stack([um * np.cos(ang), um * np.sin(ang)], 1)
    dt = 0.15 * (0.1 / 11) / I.C_LIGHT  # leapfrog limit is c dt / h ~ 0.27 here
    sp = (-I.E_CHARGE, I.M_E, 1e9, tri, lam, u)
    sim = _sim(oracle_lib, m, [sp], dt=dt, spai_level=1, bz_ext=0.05)
    free = sim.T.node_free.astype(bool)
    q0, s0 = _charge_and_div(sim)
    qprev = q0
    worst_dce = 0.0
    for step in range(40):
        sim.step(1, pusher)
        q, s = _charge_and_div(sim)
        dce = (q - qprev) + sim.dt * sim.T.divergence(sim.last_cur)
        scale = max(np.abs(q).max(), np.abs(qprev).max())
        worst_dce = max(worst_dce, np.abs(dce[free]).max() / scale)
        qprev = q
    gauss = (s - s0) - (q - q0)
    scale = max(np.abs(q).max(), np.abs(q0).max())
    assert sim.lost > 100 and sim.segments > 40 * 2000
    assert worst_dce < 1e-13
    assert np.abs(gauss[free]).max() / scale < 1e-12


def test_gauss_pair_plasma_torus(oracle_lib):
    """Self-consistent pair plasma on a torus (all nodes free): Gauss's law
    S~ d^n = q^n holds to rounding over a few hundred steps; q^0 = 0 for
    collocated pairs, so d^0 = 0 is consistent."""
    w = I.pair_plasma(n_side=10, length=0.02, n_pairs=4000, theta=0.5, steps=300)
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    sim = _sim(oracle_lib, w.mesh, sp, dt=w.dt, spai_level=1, bz_ext=w.bz_ext)
    q0 = sim.charge()
    # collocated pairs: q^0 vanishes up to the rounding of its node sums
    assert np.abs(q0).max() <= 1e-12 * abs(w.species[0].q * w.species[0].w)
    worst = 0.0
    for _ in range(6):
        sim.step(50, "boris")
        q = sim.charge()
        s = sim.T.divergence(sim.d)
        worst = max(worst, np.abs(s - (q - q0)).max() / np.abs(q).max())
    assert worst < 1e-12
    assert sim.segments > 300 * 8000
    WE, WB, WK = sim.energies()
    assert WE > 0 and WK > 0


def test_exact_inverse_gauss_literal(oracle_lib):
    """With the exact inverse of [*eps] the literal form of eq.
    semi.dis.div.2, S~ [*eps] e^n = q^n - q^0 (+ S~ [*eps] e^0), holds."""
    m = I.grid_mesh(8, 8, 0.05, 0.05, seed=12)
    rng = np.random.default_rng(6)
    tri, lam = I.sample_in_triangles(m, 500, rng)
    u = rng.normal(size=(500, 2)) * 0.3 * I.C_LIGHT
    dt = 0.2 * (0.05 / 7) / I.C_LIGHT
    sim = _sim(oracle_lib, m, [(-I.E_CHARGE, I.M_E, 1e8, tri, lam, u)], dt=dt, spai_level=-1,
               bz_ext=0.1)
    q0 = sim.charge()
    sim.step(60, "hc")
    q = sim.charge()
    Me = oracle_lib.csr_to_dense(sim.T.ne, *sim.Meps)
    free_e = sim.T.edge_free.astype(bool)
    lhs = sim.T.divergence(np.where(free_e, Me @ sim.e, 0.0))
    free = sim.T.node_free.astype(bool)
    r = lhs - (q - q0)
    assert np.abs(r[free]).max() / np.abs(q).max() < 1e-11


def test_absorbing_layer_gauss_and_loss(oracle_lib):
    """The conduction loss of the absorbing layer: with it, field energy
    injected by a particle burst decays instead of ringing in the cavity,
    and Gauss's law still holds at every node away from lossy edges."""
    w = I.large_run(n_side=30, n_particles=4000, grade=3.0)
    sp = w.species[0]
    runs = {}
    for lossy in (False, True):
        sim = oracle_lib.OracleSim(w.mesh, w.dt, [(sp.q, sp.m, sp.w * 1e-3, sp.tri, sp.lam, sp.u)],
                                   I.EPS0, I.MU0, I.C_LIGHT, spai_level=1, bz_ext=w.bz_ext)
        keep = sim.T.node_free.astype(bool)
        if lossy:
            damp, damp_b, keep = oracle_lib.absorber_damp(sim.T, w.extra["sigma_tri"], w.dt,
                                                          I.EPS0)
            sim.damp = np.ascontiguousarray(damp)
            sim.damp_b = np.ascontiguousarray(damp_b)
            assert damp.min() < 1.0 and damp.max() == 1.0
            assert damp_b.min() < 1.0 and damp_b.max() == 1.0
        q0, s0 = sim.charge(), sim.T.divergence(sim.d)
        sim.step(200, "hc")
        q, s = sim.charge(), sim.T.divergence(sim.d)
        r = (s - s0) - (q - q0)
        assert np.abs(r[keep]).max() <= 1e-12 * max(np.abs(q).max(), np.abs(q0).max())
        runs[lossy] = sim.energies()[0] + sim.energies()[1]
    assert runs[True] < runs[False]
