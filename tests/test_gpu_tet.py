"""Parity of the tetrahedral HIP path (through the C-ABI of fetd3.h) with
the FP64 tetrahedral oracle.

Tetrahedron ownership, slots and lost sets bit-exact; barycentrics and
momenta within 1e-12 (relative to their scale); e, d, b within 1e-11
relative after the run; Gauss residual and S b at rounding level."""
import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I
from paper_1707_04333_amd import inputs3 as J

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O3(oracle_lib):
    from oracle import tet
    return tet


def _g(w, level=1, **kw):
    from paper_1707_04333_amd import fetd3
    return fetd3.from_workload3(w, spai_level=level, **kw)


def _o(O3, w, level=1):
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    return O3.OracleSim3(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=level,
                         b_ext=w.extra.get("b_ext"))


def _compare_particles(osim, g, tol=1e-12):
    for si, s in enumerate(osim.species):
        gp = g.particles(si)
        alive = np.nonzero(s.tet >= 0)[0]
        assert np.array_equal(gp["id"], alive), "lost sets differ"
        assert np.array_equal(gp["tet"], s.tet[alive]), "ownership differs"
        assert np.array_equal(gp["slot"], s.slot[alive])
        assert np.abs(gp["lam"] - s.lam[alive]).max(initial=0.0) <= tol
        us = max(1.0, float(np.abs(s.u).max()))
        assert np.abs(gp["u"] - s.u[alive]).max(initial=0.0) <= tol * us


def _compare_fields(osim, g, tol=1e-11):
    for name, ref in (("e", osim.e), ("d", osim.d), ("b", osim.b)):
        got = g.field(name)
        scale = max(float(np.abs(ref).max()), 1e-300)
        assert np.abs(got - ref).max() <= tol * scale, name


def test_tet_tables_and_spai_match(O3):
    w = J.tet_pair_plasma(n_side=5, length=0.005, n_pairs=10)
    g = _g(w)
    osim = _o(O3, w)
    T = osim.T
    assert np.array_equal(g.field("edges").reshape(-1, 2), np.stack([T.edge_lo, T.edge_hi], 1))
    assert np.array_equal(g.field("faces").reshape(-1, 3), T.face_node)
    gptr, gcol, gval = g.field("spai_ptr"), g.field("spai_col"), g.field("spai_val")
    optr, ocol, oval = osim.Mt
    assert np.array_equal(gptr, optr) and np.array_equal(gcol, ocol)
    assert np.abs(gval - oval).max() <= 1e-12 * np.abs(oval).max()
    d = g.diagnostics()
    assert (d["n_edges"], d["n_faces"], d["n_tets"]) == (T.ne, T.nf, T.nt)
    g.close()


@pytest.mark.parametrize("pusher", ["boris", "boris_tan", "vay", "hc"])
def test_tet_cyclotron_parity(O3, pusher):
    w = J.tet_cyclotron(n_particles=24)
    g = _g(w)
    osim = _o(O3, w)
    osim.step(150, pusher)
    g.step(150, pusher)
    _compare_particles(osim, g)
    _compare_fields(osim, g)
    d = g.diagnostics()
    assert d["gauss_rel"] <= 1e-12 and d["divb_rel"] <= 1e-13
    g.close()


def test_tet_pair_plasma_parity_across_sorts(O3):
    w = J.tet_pair_plasma(n_side=6, length=0.006, n_pairs=3001, theta=0.3)
    g = _g(w, resort_every=7)
    osim = _o(O3, w)
    osim.step(40, "boris")
    g.step(40, "boris")
    _compare_particles(osim, g)
    _compare_fields(osim, g)
    d = g.diagnostics()
    assert d["gauss_rel"] <= 1e-12 and d["divb_rel"] <= 1e-13
    assert d["n_segments"] == osim.segments
    WE, WB, WK = osim.energies()
    assert abs(d["W_B"] - WB) <= 1e-10 * WB and abs(d["W_kin"] - WK) <= 1e-12 * WK
    g.close()


def test_tet_wall_losses_parity(O3):
    m = J.box_mesh(6, 6, 6, 0.1, 0.1, 0.1)
    rng = np.random.default_rng(6)
    n = 1500
    tet, lam = J.sample_in_tets(m, n, rng)
    gm = rng.uniform(1.2, 4.0, n)
    u = I.C_LIGHT * np.sqrt(gm * gm - 1)[:, None] * J.isotropic_directions(n, rng)
    sp = I.Species("electron", -I.E_CHARGE, I.M_E, 1e7, tet, lam, u)
    w = I.Workload("tet_walls", m, [sp], 0.1 * (0.1 / 5) / I.C_LIGHT, 30, "hc", "fp64",
                   extra={"b_ext": np.array([0.02, 0.01, 0.05])})
    g = _g(w)
    osim = _o(O3, w)
    osim.step(30, "hc")
    g.step(30, "hc")
    _compare_particles(osim, g)
    _compare_fields(osim, g)
    d = g.diagnostics()
    assert d["n_lost"] == osim.lost > 50
    assert d["gauss_rel"] <= 1e-12
    g.close()


def test_tet_fields_load_and_field_only_run(O3):
    """A field-only PEC cube seeded with b = C e (a cavity mode shape):
    100 steps match the oracle and S b stays at rounding."""
    m = J.box_mesh(7, 7, 7, 1.0, 1.0, 1.0, jitter=0.1)
    w = I.Workload("tet_cavity", m, [], 0.1 / 6 / I.C_LIGHT, 100, "boris", "fp64")
    osim = _o(O3, w)
    T = osim.T
    v = T.vxyz.reshape(-1, 4, 3)
    ez = np.zeros(T.ne)
    for k in range(6):
        p, q = O3.LE[k]
        mid = 0.5 * (v[:, p] + v[:, q])
        f = np.sin(np.pi * mid[:, 0]) * np.sin(np.pi * mid[:, 1])
        ez[T.tet_edge[:, k]] = T.tet_esign[:, k] * f * (v[:, q, 2] - v[:, p, 2])
    ez[~T.edge_free.astype(bool)] = 0.0
    b0 = T.curl(ez) * 1e-9
    g = _g(w)
    g.fields_load(b=b0)
    assert np.array_equal(g.field("b"), b0)
    osim.b = b0.copy()
    osim.step(100)
    g.step(100)
    _compare_fields(osim, g)
    d = g.diagnostics()
    assert d["divb_rel"] <= 1e-12
    g.close()


def test_tet_error_paths():
    from paper_1707_04333_amd import fetd3
    from paper_1707_04333_amd.fetdpic import FETD_E_TRACK, FetdError
    w = J.tet_cyclotron(n_particles=8)
    g = fetd3.from_workload3(w, crossing_cap=1)
    g.step(100, "boris")
    with pytest.raises(FetdError) as ei:
        g.sync()
    assert ei.value.status == FETD_E_TRACK
    g.close()
    s = w.species[0]
    g = _g(I.Workload("x", w.mesh, [], w.dt, 1, "boris", "fp64", extra=w.extra))
    u = s.u.copy()
    u[2, 1] = np.nan
    g.load(s.q, s.m, s.w, s.tri, s.lam, u)
    g.step(2, "boris")
    with pytest.raises(FetdError) as ei:
        g.sync()
    assert ei.value.status == FETD_E_TRACK
    g.close()


def _percentile_errors3(osim, g):
    el, eu, mis, total = [], [], 0, 0
    us = max(float(np.abs(s.u).max()) for s in osim.species)
    for si, s in enumerate(osim.species):
        gp = g.particles(si)
        alive = np.nonzero(s.tet >= 0)[0]
        assert np.array_equal(gp["id"], alive), "lost sets differ"
        same = (gp["tet"] == s.tet[alive]) & (gp["slot"] == s.slot[alive])
        mis += int((~same).sum())
        total += alive.size
        el.append(np.abs(gp["lam"][same] - s.lam[alive][same]).max(axis=1))
        eu.append(np.abs(gp["u"][same] - s.u[alive][same]).max(axis=1) / us)
    el, eu = np.concatenate(el), np.concatenate(eu)
    return mis, total, np.percentile(el, [50, 99, 100]), np.percentile(eu, [50, 99, 100])


def test_tet_mixed_precision_gauss_and_error(O3):
    """Mixed mode (FP32 particle state, gather, push and march; FP64
    barycentrics in flight, deposit and fields) against the FP64 oracle:
    Gauss's law and S b stay at FP64 rounding; without self-fields every
    particle agrees to FP32 accuracy; with them the bulk (99th percentile)
    and the kinetic energy are bounded."""
    w = J.tet_pair_plasma(n_side=8, length=0.008, n_pairs=20_000, theta=0.3)
    weak = J.tet_pair_plasma(n_side=8, length=0.008, n_pairs=20_000, theta=0.3)
    for s in weak.species:
        s.w = 1e-6
    for wl, tol in ((weak, None), (w, 1e-4)):
        osim = _o(O3, wl)
        g = _g(wl, precision="mixed", resort_every=9)
        osim.step(30, "boris")
        g.step(30, "boris")
        d = g.diagnostics()
        assert d["gauss_rel"] <= 1e-12 and d["divb_rel"] <= 1e-13, d
        mis, total, el, eu = _percentile_errors3(osim, g)
        assert mis <= 1e-3 * total, mis
        if tol is None:
            assert el[2] <= 2e-5 and eu[2] <= 2e-6, (el, eu)
        else:
            assert el[1] <= tol and eu[1] <= tol, (el, eu)
            assert abs(d["W_kin"] / osim.energies()[2] - 1) < 1e-4
        g.close()
