"""Parity at the benchmark's sizes and launch shapes, and the particle
kernel's rarely taken branches, through the C-ABI against the FP64 oracle.

* The 16M-particle pair plasma (199,712 triangles; 7,813 blocks of 1,024
  particles per species launch) at kT/mc^2 = 0.1 and 1: three FP64 steps
  over all particles against the oracle (its threaded timing mode, whose
  particle arithmetic is the parity mode's; pinned to it on the CPU), and
  the mixed precision forms against the same oracle within their bounds.
* The 128M-particle graded run of the benchmark's headline (1.0M
  triangles, 125,000 blocks): its first FP64 step moves every particle in
  the applied field only (the self-field starts at zero), so each sampled
  particle's step is the oracle's single-particle step; Gauss's law holds
  over the whole mesh.
* More than 384 (FP64) or 512 (FP32) of a 1,024-particle tile's particles
  leaving their triangle in one step overflow the kernel's LDS crossing
  queue; the overflow is finished in place (in FP64 from the start state,
  as phase 2 does).  A run where about 95% of the particles cross edges
  every step checks that branch against the oracle.
"""
import os

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def _fp():
    from paper_1707_04333_amd import fetdpic
    return fetdpic


def _oracle_sim(oracle_lib, w, level=1):
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    return oracle_lib.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=level,
                                bz_ext=(w.bz_ext if w.bz_ext else None), affine=w.e_affine)


def _compare_fp64(osim, g, field_tol=1e-11):
    """Ownership, slot and lost sets bit-exact; barycentrics and momenta to
    1e-12; fields to field_tol of their scale."""
    for si, s in enumerate(osim.species):
        gp = g.particles(si)
        alive = np.nonzero(s.tri >= 0)[0]
        assert np.array_equal(gp["id"], alive), "lost sets differ"
        same = (gp["tri"] == s.tri[alive]) & (gp["slot"] == s.slot[alive])
        assert same.all(), f"{int((~same).sum())} ownership mismatches"
        assert np.abs(gp["lam"] - s.lam[alive]).max() <= 1e-12
        us = max(1.0, float(np.abs(s.u).max()))
        assert np.abs(gp["u"] - s.u[alive]).max() <= 1e-12 * us
    for name, ref in (("e", osim.e), ("d", osim.d), ("b", osim.b)):
        got = g.field(name)
        scale = max(float(np.abs(ref).max()), 1e-300)
        assert float(np.abs(got - ref).max()) <= field_tol * scale, name


@pytest.mark.timeout(600)
@pytest.mark.parametrize("theta", [0.1, 1.0])
def test_full_size_pair_plasma_parity(oracle_lib, theta):
    fp = _fp()
    print(f"[full-size pair plasma theta={theta}]", flush=True)
    w = I.pair_plasma(theta=theta, precision="fp64")
    assert w.n_particles == 16_000_000 and w.mesh.n_tris == 199_712
    osim = _oracle_sim(oracle_lib, w)
    g = fp.from_workload(w, precision="fp64", spai_level=1)
    for _ in range(3):
        osim.step(1, "boris", threads=THREADS)
    g.step(3, "boris")
    _compare_fp64(osim, g)
    d = g.diagnostics()
    assert d["gauss_rel"] <= 1e-12 and d["n_segments"] == osim.segments
    g.close()
    # both mixed forms against the FP64 oracle after the same three steps
    for prec in ("mixed", "mixed_f64field"):
        gm = fp.from_workload(w, precision=prec, spai_level=1)
        gm.step(3, "boris")
        dm = gm.diagnostics()
        assert dm["gauss_rel"] <= 1e-6, (prec, dm["gauss_rel"])
        mis = total = 0
        el, eu = [], []
        us = max(float(np.abs(s.u).max()) for s in osim.species)
        for si, s in enumerate(osim.species):
            gp = gm.particles(si)
            alive = np.nonzero(s.tri >= 0)[0]
            same = (gp["tri"] == s.tri[alive]) & (gp["slot"] == s.slot[alive])
            mis += int((~same).sum())
            total += alive.size
            el.append(np.abs(gp["lam"][same] - s.lam[alive][same]).max(axis=1))
            eu.append(np.abs(gp["u"][same] - s.u[alive][same]).max(axis=1) / us)
        el, eu = np.concatenate(el), np.concatenate(eu)
        # FP32 state: a few ulp of FP32 per step; ownership differs only for
        # particles within FP32 rounding of an edge
        assert mis <= 1e-4 * total, (prec, mis)
        assert np.percentile(el, 99) <= 1e-5 and np.percentile(eu, 99) <= 1e-5, prec
        WE, WB, WK = osim.energies()
        assert abs(dm["W_kin"] / WK - 1.0) < 1e-5, prec
        gm.close()


@pytest.mark.timeout(600)
def test_full_size_graded_run_first_step(oracle_lib):
    """The 128M-electron graded run with its absorbing layer (FP64, HC):
    one step; 200,000 sampled particles against the oracle's step of the
    same particles in the applied field (e = 0, b = 0 at step 0, so each
    particle's first step is independent of all others)."""
    fp = _fp()
    print("[full-size graded run, 128M electrons]", flush=True)
    w = I.large_run(precision="fp64")
    assert w.n_particles == 128_000_000
    sp = w.species[0]
    g = fp.from_workload(w, precision="fp64", spai_level=1)
    g.diagnostics()
    g.step(1, "hc")
    d = g.diagnostics()
    assert d["gauss_rel"] <= 1e-12 and d["error_code"] == 0
    got = g.particles(0)
    rng = np.random.default_rng(77)
    pick = np.sort(rng.choice(sp.n, 200_000, replace=False))
    sub = I.Species("sample", sp.q, sp.m, sp.w, sp.tri[pick], sp.lam[pick], sp.u[pick])
    ws = I.Workload("sample", w.mesh, [sub], w.dt, 1, "hc", "fp64", bz_ext=w.bz_ext,
                    spai_level=1)
    osim = _oracle_sim(oracle_lib, ws)
    damp, damp_b, _ = oracle_lib.absorber_damp(osim.T, w.extra["sigma_tri"], w.dt, I.EPS0)
    osim.damp, osim.damp_b = np.ascontiguousarray(damp), np.ascontiguousarray(damp_b)
    osim.step(1, "hc")
    s = osim.species[0]
    alive_o = s.tri >= 0
    # the library returns the alive particles in load order with their ids
    pos = np.searchsorted(got["id"], pick)
    found = (pos < got["id"].size) & (got["id"][np.minimum(pos, got["id"].size - 1)] == pick)
    assert np.array_equal(found, alive_o), "lost sets differ"
    pos = pos[found]
    assert np.array_equal(got["tri"][pos], s.tri[alive_o])
    assert np.array_equal(got["slot"][pos], s.slot[alive_o])
    assert np.abs(got["lam"][pos] - s.lam[alive_o]).max() <= 1e-12
    assert np.abs(got["u"][pos] - s.u[alive_o]).max() <= 1e-12 * np.abs(s.u).max()
    g.close()


def _crossing_workload(n_pairs=20_011):
    """Hot pair plasma (kT/mc^2 = 3) stepped with c dt = 2.5 h, so a particle
    moves up to 2.5 cells per step and about 95% leave their triangle; the
    weight is cut by 1e6 (negligible self-field: the step is far past the
    field update's stability limit, which only matters for the fields'
    size, compared relative to their own scale)."""
    w = I.pair_plasma(n_side=16, length=0.025, n_pairs=n_pairs, theta=3.0, steps=4,
                      precision="fp64")
    w.dt = 2.5 * (0.025 / 16) / I.C_LIGHT
    for s in w.species:
        s.w *= 1e-6
    return w


@pytest.mark.parametrize("deterministic", [False, True])
def test_crossing_queue_overflow_parity(oracle_lib, deterministic):
    fp = _fp()
    w = _crossing_workload()
    osim = _oracle_sim(oracle_lib, w)
    g = fp.from_workload(w, precision="fp64", spai_level=1, deterministic=deterministic,
                         resort_every=2)
    for step in range(4):
        before = [s.tri.copy() for s in osim.species]
        osim.step(1, "boris")
        g.step(1, "boris")
        left = sum(int((b != s.tri).sum()) for b, s in zip(before, osim.species))
        # every tile of 1024 holds far more leavers than the queue's 384 entries
        assert left > 0.85 * w.n_particles, left
        _compare_fp64(osim, g, field_tol=1e-10)
    g.close()
