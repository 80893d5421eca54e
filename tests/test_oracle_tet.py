"""Pins of the tetrahedral oracle (Sec. II in three dimensions) against
what the mathematics fixes:

  * topology: Euler characteristic (1 for a box, 0 for a periodic one),
    S C = 0 and C G = 0 exactly on integer vectors (the discrete
    div-curl and curl-grad identities behind eqs. semi.dis.div.1/2),
    opposite outward signs of a face in its two tetrahedra, node identity
    across faces;
  * Whitney forms: the line integral of W1_k along edge l and the flux of
    W2_k through face l are delta_kl; curl (sum e W1) = sum (C e) W2 and
    div (sum b W2) = (S b)/V by finite differences (both sides are linear
    in a tetrahedron, so central differences are exact to rounding);
    uniform fields are reproduced exactly and the Hodge matrices give their
    energies (eps0 |E|^2 V, |B|^2 V / mu0);
  * scatter: the current of one piece is the exact line integral of W1 and
    its dipole moment sum_e i_e t_e is Q dr / dt;
  * the run: continuity at every free node and step, Gauss's law and
    S b = 0 over whole runs with wall losses and on a 3-torus; the Boris
    orbit in a uniform B keeps |u| and u.B; a PEC cavity rings at its
    lowest eigenfrequency c pi sqrt(1/a^2 + 1/b^2) (mesh error O(h^2))."""
import math

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I
from paper_1707_04333_amd import inputs3 as J


@pytest.fixture(scope="module")
def O3(oracle_lib):
    from oracle import tet
    return tet


def _topo(O3, per=(False, False, False), n=(5, 4, 4)):
    m = J.box_mesh(*n, 1.0, 0.8, 0.9, periodic=per)
    return m, O3.Topology3(m.node_xyz, m.tet_nodes, m.tet_shift, m.period)


@pytest.mark.parametrize("per,chi", [((False,) * 3, 1), ((True,) * 3, 0), ((True, False, True), 0)])
def test_topology_identities(O3, per, chi):
    m, T = _topo(O3, per)
    assert T.nn - T.ne + T.nf - T.nt == chi
    rng = np.random.default_rng(1)
    e = rng.integers(-50, 50, T.ne).astype(np.float64)
    assert np.all(T.face_divergence(T.curl(e)) == 0.0)
    phi = rng.integers(-50, 50, T.nn).astype(np.float64)
    assert np.all(T.curl(phi[T.edge_hi] - phi[T.edge_lo]) == 0.0)
    two = T.face_tet[:, 1] >= 0
    s0 = T.tet_fout[T.face_tet[two, 0], T.face_tk[two, 0]]
    s1 = T.tet_fout[T.face_tet[two, 1], T.face_tk[two, 1]]
    assert np.all(s0 == -s1)
    # node identity across every face
    for t in range(T.nt):
        for k in range(4):
            nb = T.tet_nbr[t, k]
            if nb < 0:
                continue
            mp = T.tet_nbrmap[t].reshape(4, 4)[k]
            for j in range(4):
                if j != k:
                    assert T.tet_node[nb, mp[j]] == T.tet_node[t, j]
            assert T.tet_nbr[nb, mp[k]] == t
    if per == (True,) * 3:
        assert T.edge_free.all() and T.node_free.all()


def _sim(O3, m, species=(), **kw):
    return O3.OracleSim3(m, kw.pop("dt", 1e-12), list(species), I.EPS0, I.MU0, I.C_LIGHT, **kw)


def test_whitney_dofs_are_kronecker(O3):
    m, T = _topo(O3, (True, False, False))
    sim = _sim(O3, m)
    v = T.vxyz.reshape(-1, 4, 3)
    for t in range(0, T.nt, 7):
        # W1 of every local edge along every local edge
        for l in range(6):
            a, b = O3.LE[l]
            L = np.zeros(4)
            L[a] = L[b] = 0.5
            tvec = v[t, b] - v[t, a]
            for k in range(6):
                e = np.zeros(T.ne)
                e[T.tet_edge[t, k]] = T.tet_esign[t, k]  # W1 of local edge k, local orientation
                E, _ = O3.gather3(sim, t, L, e=e)
                assert abs(E @ tvec - (1.0 if k == l else 0.0)) <= 1e-12
        # W2 of every local face through every local face
        for l in range(4):
            p, q, r = O3.LF[l]
            L = np.zeros(4)
            L[[p, q, r]] = 1.0 / 3.0
            area = 0.5 * np.cross(v[t, q] - v[t, p], v[t, r] - v[t, p])
            for k in range(4):
                b = np.zeros(T.nf)
                b[T.tet_face[t, k]] = T.tet_fpar[t, k]  # local sorted orientation
                _, B = O3.gather3(sim, t, L, b=b)
                assert abs(B @ area - (1.0 if k == l else 0.0)) <= 1e-12


def _inside_point(rng):
    L = rng.dirichlet([4, 4, 4, 4])
    return L


def test_curl_and_divergence_of_whitney_fields(O3):
    m, T = _topo(O3, (False, True, False))
    sim = _sim(O3, m)
    rng = np.random.default_rng(3)
    e = rng.normal(size=T.ne)
    b = rng.normal(size=T.nf)
    Ce = T.curl(e)
    Sb = T.face_divergence(b)
    v = T.vxyz.reshape(-1, 4, 3)
    G = T.grad.reshape(-1, 4, 3)
    h = 1e-3
    for t in rng.choice(T.nt, 40, replace=False):
        L0 = _inside_point(rng)
        jac_e = np.zeros((3, 3))
        jac_b = np.zeros((3, 3))
        for x in range(3):
            dL = G[t, :, x] * h  # barycentric change for a step h along axis x
            Ep, Bp = O3.gather3(sim, t, L0 + dL, e=e, b=b)
            Em, Bm = O3.gather3(sim, t, L0 - dL, e=e, b=b)
            jac_e[:, x] = (Ep - Em) / (2 * h)
            jac_b[:, x] = (Bp - Bm) / (2 * h)
        curl = np.array([jac_e[2, 1] - jac_e[1, 2], jac_e[0, 2] - jac_e[2, 0],
                         jac_e[1, 0] - jac_e[0, 1]])
        _, Bc = O3.gather3(sim, t, L0, e=e, b=Ce)
        assert np.abs(curl - Bc).max() <= 1e-8 * max(1.0, np.abs(Bc).max())
        div = np.trace(jac_b)
        assert abs(div - Sb[t] / T.vol[t]) <= 1e-8 * abs(Sb[t] / T.vol[t]) + 1e-6


def test_uniform_fields_and_hodge_energies(O3):
    m, T = _topo(O3, (True, True, True))
    sim = _sim(O3, m)
    E0 = np.array([0.3, -1.2, 0.7])
    B0 = np.array([-0.4, 0.25, 1.1])
    xyz = m.node_xyz
    # line integrals along image-consistent edge vectors (from any tetrahedron)
    tvec = np.zeros((T.ne, 3))
    v = T.vxyz.reshape(-1, 4, 3)
    for k in range(6):
        a, b = O3.LE[k]
        tvec[T.tet_edge[:, k]] = T.tet_esign[:, k, None] * (v[:, b] - v[:, a])
    e = tvec @ E0
    avec = np.zeros((T.nf, 3))
    for k in range(4):
        p, q, r = O3.LF[k]
        avec[T.tet_face[:, k]] = T.tet_fpar[:, k, None] * 0.5 * np.cross(v[:, q] - v[:, p],
                                                                       v[:, r] - v[:, p])
    b = avec @ B0
    rng = np.random.default_rng(4)
    for t in rng.choice(T.nt, 30, replace=False):
        E, B = O3.gather3(sim, t, rng.dirichlet([1, 1, 1, 1]), e=e, b=b)
        assert np.abs(E - E0).max() <= 1e-12 and np.abs(B - B0).max() <= 1e-12
    from oracle import csr_matvec
    vol = T.vol.sum()
    assert abs(e @ csr_matvec(*sim.Meps, e) - I.EPS0 * (E0 @ E0) * vol) <= 1e-12 * I.EPS0 * vol
    assert abs(b @ csr_matvec(*sim.Mnu, b) - (B0 @ B0) * vol / I.MU0) <= 1e-12 * vol / I.MU0
    assert np.abs(T.face_divergence(b)).max() <= 1e-15
    assert xyz.shape[1] == 3


def test_segment_current_exact_and_dipole(O3):
    m, T = _topo(O3, (False, False, False), n=(7, 7, 7))
    sim = _sim(O3, m)
    v = T.vxyz.reshape(-1, 4, 3)
    G = T.grad.reshape(-1, 4, 3)
    tvec = np.zeros((T.ne, 3))
    for k in range(6):
        a, b = O3.LE[k]
        tvec[T.tet_edge[:, k]] = T.tet_esign[:, k, None] * (v[:, b] - v[:, a])
    rng = np.random.default_rng(5)
    cen = v.mean(axis=1)
    inner = np.nonzero(np.all((cen > 0.3) & (cen < 0.6), axis=1))[0]
    for _ in range(40):
        t = int(rng.choice(inner))
        Ls = rng.dirichlet([2, 2, 2, 2])
        Lf = rng.dirichlet([2, 2, 2, 2])
        dr = (Lf - Ls) @ v[t]
        t2, s2, p2, lost, ns, cur = O3.move3(sim, t, 0, Ls[1:], dr)
        assert ns == 1 and t2 == t and not lost
        Lm = 0.5 * (Ls + Lf)
        for k in range(6):
            a, b = O3.LE[k]
            W = Lm[a] * G[t, b] - Lm[b] * G[t, a]
            assert abs(cur[T.tet_edge[t, k]] - T.tet_esign[t, k] * (W @ dr)) <= 1e-14
        # a long move through many tetrahedra
        ang = rng.normal(size=3)
        d = rng.uniform(0.05, 0.2) * ang / np.linalg.norm(ang)
        t3, s3, p3, lost, ns, cur = O3.move3(sim, t, 0, Ls[1:], d)
        assert not lost and ns >= 1
        assert np.abs(cur @ tvec - d).max() <= 1e-13
        # two halves deposit the same current as the whole
        ta, sa, pa, _, _, ca = O3.move3(sim, t, 0, Ls[1:], d / 2)
        _, _, _, _, _, cb = O3.move3(sim, ta, sa, pa, d / 2)
        assert np.abs(ca + cb - cur).max() <= 1e-14


@pytest.mark.parametrize("pusher", ["boris", "vay", "hc", "boris_tan"])
def test_continuity_gauss_and_divb_with_wall_losses(O3, pusher):
    m = J.box_mesh(6, 6, 6, 0.1, 0.1, 0.1)
    rng = np.random.default_rng(6)
    n = 1500
    tet, lam = J.sample_in_tets(m, n, rng)
    g = rng.uniform(1.2, 4.0, n)
    u = I.C_LIGHT * np.sqrt(g * g - 1)[:, None] * J.isotropic_directions(n, rng)
    dt = 0.1 * (0.1 / 5) / I.C_LIGHT
    sim = _sim(O3, m, [(-I.E_CHARGE, I.M_E, 1e7, tet, lam, u)], dt=dt, spai_level=1,
               b_ext=np.array([0.02, 0.01, 0.05]))
    free = sim.T.node_free.astype(bool)
    q0 = sim.charge()
    s0 = sim.T.divergence(sim.d)
    qprev = q0
    worst = 0.0
    for _ in range(30):
        sim.step(1, pusher)
        q = sim.charge()
        dce = (q - qprev) + sim.dt * sim.T.divergence(sim.last_cur)
        worst = max(worst, np.abs(dce[free]).max() / max(np.abs(q).max(), np.abs(qprev).max()))
        qprev = q
    s = sim.T.divergence(sim.d)
    gauss = (s - s0) - (q - q0)
    assert sim.lost > 50 and sim.segments > 30 * 1000
    assert worst < 1e-13
    assert np.abs(gauss[free]).max() / max(np.abs(q).max(), np.abs(q0).max()) < 1e-12
    assert np.abs(sim.T.face_divergence(sim.b)).max() <= 1e-13 * np.abs(sim.b).max()
    assert np.abs(sim.b).max() > 0


def test_pair_plasma_torus_gauss(O3):
    w = J.tet_pair_plasma(n_side=5, length=0.005, n_pairs=3000, theta=0.3, steps=100)
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    sim = _sim(O3, w.mesh, sp, dt=w.dt, spai_level=1, b_ext=w.extra["b_ext"])
    q0 = sim.charge()
    assert np.abs(q0).max() <= 1e-12 * abs(w.species[0].q * w.species[0].w)
    worst = 0.0
    for _ in range(4):
        sim.step(25, "boris")
        q = sim.charge()
        worst = max(worst, np.abs(sim.T.divergence(sim.d) - (q - q0)).max() / np.abs(q).max())
    assert worst < 1e-12
    assert np.abs(sim.T.face_divergence(sim.b)).max() <= 1e-12 * np.abs(sim.b).max()
    WE, WB, WK = sim.energies()
    assert WE > 0 and WB > 0 and WK > 0


def test_boris_orbit_in_uniform_b(O3):
    w = J.tet_cyclotron(n_particles=8)
    s = w.species[0]
    sim = _sim(O3, w.mesh, [(s.q, s.m, 1e-12, s.tri, s.lam, s.u)], dt=w.dt, spai_level=1,
               b_ext=w.extra["b_ext"])
    bhat = w.extra["b_ext"] / np.linalg.norm(w.extra["b_ext"])
    u0 = sim.species[0].u.copy()
    x0 = sim.positions(sim.species[0])
    sim.step(50, "boris")
    u1 = sim.species[0].u
    assert np.abs(np.linalg.norm(u1, axis=1) / np.linalg.norm(u0, axis=1) - 1).max() <= 1e-12
    assert np.abs(u1 @ bhat - u0 @ bhat).max() <= 1e-9 * np.abs(u0).max()
    # drift along B over 50 steps: dt sum of v_par
    g = np.sqrt(1 + np.sum(u0 ** 2, axis=1) / I.C_LIGHT ** 2)
    x1 = sim.positions(sim.species[0])
    par = (x1 - x0) @ bhat
    assert np.abs(par - 50 * w.dt * (u0 @ bhat) / g).max() <= 1e-9


def _crossing_frequency(x, dt):
    """Angular frequency of W_B(t) ~ cos^2(w t) from its mean crossings
    (one every pi / (2 w)), linearly interpolated."""
    x = x - x.mean()
    s = np.sign(x)
    idx = np.nonzero(s[1:] != s[:-1])[0]
    tc = np.array([(i + x[i] / (x[i] - x[i + 1])) * dt for i in idx])
    return np.pi / (2 * np.mean(np.diff(tc)))


def test_cavity_lowest_mode_frequency(O3):
    """With the exact inverse of [*eps] the discrete PEC cube rings at
    c pi sqrt(2)/a within the mesh's O(h^2) error (measured 0.1% at 7^3
    nodes); three periods, b seeded as C e of E_z = sin(pi x) sin(pi y)."""
    a = 1.0
    n = 7
    m = J.box_mesh(n, n, n, a, a, a, jitter=0.1)
    h = a / (n - 1)
    dt = 0.1 * h / I.C_LIGHT
    sim = _sim(O3, m, dt=dt, spai_level=-1)
    T = sim.T
    v = T.vxyz.reshape(-1, 4, 3)
    ez = np.zeros(T.ne)
    for k in range(6):
        p, q = O3.LE[k]
        mid = 0.5 * (v[:, p] + v[:, q])
        f = np.sin(np.pi * mid[:, 0] / a) * np.sin(np.pi * mid[:, 1] / a)
        ez[T.tet_edge[:, k]] = T.tet_esign[:, k] * f * (v[:, q, 2] - v[:, p, 2])
    ez[~T.edge_free.astype(bool)] = 0.0
    sim.b = T.curl(ez) * 1e-9
    w_exact = I.C_LIGHT * np.pi * math.sqrt(2) / a
    steps = int(3 * 2 * np.pi / w_exact / dt)
    from oracle import csr_matvec
    wb = []
    for _ in range(steps):
        sim.step(1)
        wb.append(sim.b @ csr_matvec(*sim.Mnu, sim.b))
    w_num = _crossing_frequency(np.array(wb), dt)
    assert abs(w_num / w_exact - 1) < 0.005
    assert np.abs(T.face_divergence(sim.b)).max() <= 1e-12 * np.abs(sim.b).max()
