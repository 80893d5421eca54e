"""Error of the mixed mode (FP32 particle state, gather, push and tracking;
FP64 deposit and fields) against FP64, stated per result:

- gyroradius: relativistic cyclotron orbits (64 electrons, gamma 1.5-10,
  B = 1 T), circle fits of 400 steps of the mixed GPU run against the FP64
  oracle's orbits;
- field energy: W_E and W_B of the self-consistent pair plasma after 50
  steps against the FP64 oracle's (W_E is the energy of the charge
  separation of pairs that start collocated, a noise quantity grown from
  zero: it carries the chaotic amplification of the FP32 trajectory
  differences and gets a looser bound than W_B and W_kin);
- Bernstein-mode frequency: the first-band ridge of the dispersion run
  (32,768 steps of 2.7M particles, too long for the oracle) against the
  same run in FP64 on the GPU, the path the parity tests hold to the
  oracle within 1e-12.
"""
import numpy as np
import pytest

from paper_1707_04333_amd import dispersion as D
from paper_1707_04333_amd import inputs as I

pytestmark = pytest.mark.gpu


def _circle(xy):
    """Algebraic least-squares circle: centre and radius."""
    A = np.column_stack([2 * xy[:, 0], 2 * xy[:, 1], np.ones(len(xy))])
    b = (xy ** 2).sum(axis=1)
    cx, cy, c0 = np.linalg.lstsq(A, b, rcond=None)[0]
    return cx, cy, np.sqrt(c0 + cx * cx + cy * cy)


def test_gyroradius_mixed_against_oracle(oracle_lib):
    from paper_1707_04333_amd import fetdpic as fp
    w = I.cyclotron()
    sp = w.species[0]
    osim = oracle_lib.OracleSim(w.mesh, w.dt, [(sp.q, sp.m, sp.w, sp.tri, sp.lam, sp.u)],
                                I.EPS0, I.MU0, I.C_LIGHT, spai_level=w.spai_level,
                                bz_ext=w.bz_ext)
    g = fp.from_workload(w, precision="mixed")
    n_steps = 400
    to = np.empty((n_steps + 1, sp.n, 2))
    tg = np.empty((n_steps + 1, sp.n, 2))
    to[0] = tg[0] = osim.positions(osim.species[0])
    for i in range(n_steps):
        osim.step(1, "boris")
        g.step(1, "boris")
        to[i + 1] = osim.positions(osim.species[0])
        p = g.particles(0)
        assert np.array_equal(p["id"], np.arange(sp.n))
        s = oracle_lib.OSpecies(sp.q, sp.m, sp.w, p["tri"], p["lam"], p["u"], p["slot"])
        tg[i + 1] = osim.positions(s)
    g.close()
    rel = []
    for k in range(sp.n):
        ro = _circle(to[:, k])[2]
        rg = _circle(tg[:, k])[2]
        rel.append(abs(rg / ro - 1.0))
    rel = np.array(rel)
    print(f"gyroradius, mixed vs FP64 oracle: median {np.median(rel):.2e}, max {rel.max():.2e}")
    assert rel.max() <= 1e-5


def test_field_energy_mixed_against_oracle(oracle_lib):
    from paper_1707_04333_amd import fetdpic as fp
    w = I.pair_plasma(n_side=24, length=0.038, n_pairs=20_000, theta=0.3, steps=100,
                      precision="mixed")
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = oracle_lib.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1,
                                bz_ext=w.bz_ext)
    g = fp.from_workload(w, precision="mixed", spai_level=1)
    g.diagnostics()
    osim.step(50, "boris")
    g.step(50, "boris")
    d = g.diagnostics()
    g.close()
    WE, WB, WK = osim.energies()
    eE, eB, eK = abs(d["W_E"] / WE - 1), abs(d["W_B"] / WB - 1), abs(d["W_kin"] / WK - 1)
    print(f"field energy, mixed vs FP64 oracle after 50 steps: W_E {eE:.2e}, W_B {eB:.2e}, "
          f"W_kin {eK:.2e}")
    assert eE <= 2e-2 and eB <= 1e-4 and eK <= 1e-4


def _ridge(precision):
    from paper_1707_04333_amd import fetdpic as fp
    w = I.bernstein_strip()
    sim = fp.from_workload(w, precision=precision)
    nx, every, steps = 428, 16, 32768
    lx, ly = w.extra["length_x"], w.extra["length_y"]
    xy = np.stack([(np.arange(nx) + 0.5) * lx / nx, np.full(nx, 0.5 * ly)], axis=1)
    sim.probe_set(xy, every=every, max_samples=steps // every)
    sim.set_resort(20)
    sim.step(steps, "boris")
    samples = sim.probe_get()
    sim.close()
    k, om, p = D.spectrum(samples, every * w.dt, lx / nx, w.extra["omega_c"], I.C_LIGHT)
    sel = (k > 0.9) & (k < 38.0)
    return D.ridge(k, om, p, 1)[sel], om[1] - om[0]


def test_bernstein_frequency_mixed_against_fp64():
    rm, dw = _ridge("mixed")
    r64, _ = _ridge("fp64")
    dev = np.abs(rm - r64)
    print(f"band-1 ridge, mixed vs FP64: median {np.median(dev):.4f} omega_c, "
          f"90th percentile {np.percentile(dev, 90):.4f} (resolution {dw:.4f})")
    assert np.median(dev) <= dw + 1e-12
    assert np.percentile(dev, 90) <= 3 * dw
