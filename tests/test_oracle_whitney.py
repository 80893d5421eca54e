"""Pins of the oracle's mesh, Whitney-form and Hodge machinery (Sec. II.A-B).

What fixes the answer here is the mathematics of lowest-order Whitney
forms: edge elements reproduce every field of the form a + w z x r exactly,
face elements reproduce uniform B exactly, the incidence matrices satisfy
C G = 0 in integers, the Euler characteristic of the mesh is topological,
and [*eps] is the SPD Gram matrix of the W1 basis (so e^T [*eps] e of a
uniform field is eps0 |E|^2 times the area)."""
import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _topo(oracle_lib, *args, **kw):
    m = I.grid_mesh(*args, **kw)
    return m, oracle_lib.Topology(m.node_xy, m.tri_nodes, m.tri_shift, m.period)


def _sim(oracle_lib, m, level=1):
    return oracle_lib.OracleSim(m, 1e-12, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=level)


def _edge_vec(T):
    """Edge vector lo -> hi in the frame of the first adjacent triangle."""
    f = T.edge_tri[:, 0]
    v = T.vxy.reshape(-1, 3, 2)
    out = np.zeros((T.ne, 2))
    start = np.zeros((T.ne, 2))
    for e in range(T.ne):
        k = np.nonzero(T.tri_edge[f[e]] == e)[0][0]
        a, b = (k + 1) % 3, (k + 2) % 3
        pa, pb = v[f[e], a], v[f[e], b]
        if T.tri_sign[f[e], k] > 0:
            start[e], out[e] = pa, pb - pa
        else:
            start[e], out[e] = pb, pa - pb
    return start, out


@pytest.mark.parametrize("args,chi", [((9, 7, 1.0, 0.8), 1),
                                      ((33, 33, 1.0, 1.0), 1),
                                      ((10, 9, 1.0, 1.0, True, False), 0),
                                      ((8, 11, 0.5, 0.5, True, True), 0)])
def test_topology_invariants(oracle_lib, args, chi):
    """Euler characteristic N_n - N_e + N_f (1 for a disk, 0 for an annulus
    or torus; the paper's Bernstein mesh has 7252 - 18123 + 10872 = 1) and
    C G = 0 in integers (curl of a gradient vanishes)."""
    m, T = _topo(oracle_lib, *args)
    assert T.nn - T.ne + T.nf == chi
    # integer-valued matrices held in float64: the products are exact
    C = np.zeros((T.nf, T.ne))
    r, c, v = T.curl_matrix()
    C[r, c] = v
    G = np.zeros((T.ne, T.nn))
    r, c, v = T.grad_matrix()
    G[r, c] = v
    assert not np.any(C @ G)
    assert set(np.unique(C)) <= {-1, 0, 1}
    # every interior edge is traversed once in each direction by its faces
    two = T.edge_tri[:, 1] >= 0
    assert np.all(T.edge_tsign[two, 0] == -T.edge_tsign[two, 1])
    # S~ = -G^T: the divergence of a gradient's dual is the graph Laplacian
    x = np.random.default_rng(0).normal(size=T.ne)
    assert np.allclose(T.divergence(x), -(G.T @ x))


def test_uniform_and_rotational_field_reproduced(oracle_lib):
    """E = a + w z x r has line-integral DoFs e = a . dl + w (p x q) on the
    straight edge p -> q; its Whitney interpolant is exact (Sec. II.B)."""
    m, T = _topo(oracle_lib, 9, 8, 1.0, 0.9)
    sim = _sim(oracle_lib, m)
    start, dl = _edge_vec(T)
    q = start + dl
    a = np.array([3.5, -1.25])
    w = 0.75
    e = dl @ a + w * (start[:, 0] * q[:, 1] - start[:, 1] * q[:, 0])
    rng = np.random.default_rng(3)
    v = T.vxy.reshape(-1, 3, 2)
    for _ in range(200):
        f = int(rng.integers(T.nf))
        L = rng.dirichlet([1, 1, 1])
        E = oracle_lib.gather_e(sim, f, L, e)
        r = L @ v[f]
        ref = a + w * np.array([-r[1], r[0]])
        assert np.abs(E - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tangential_continuity(oracle_lib):
    """The tangential component of a W1 interpolant is continuous across an
    interior edge: both triangles see the same E . t at a shared point."""
    m, T = _topo(oracle_lib, 8, 8, 1.0, 1.0)
    sim = _sim(oracle_lib, m)
    rng = np.random.default_rng(4)
    e = rng.normal(size=T.ne)
    v = T.vxy.reshape(-1, 3, 2)
    for ed in np.nonzero(T.edge_tri[:, 1] >= 0)[0][:100]:
        s = rng.random()
        vals = []
        for j in range(2):
            f = T.edge_tri[ed, j]
            k = int(np.nonzero(T.tri_edge[f] == ed)[0][0])
            a, b = (k + 1) % 3, (k + 2) % 3
            L = np.zeros(3)
            # point at fraction s from the edge's low node to its high node
            if T.tri_sign[f, k] > 0:
                L[a], L[b] = 1 - s, s
                t = v[f, b] - v[f, a]
            else:
                L[b], L[a] = 1 - s, s
                t = v[f, a] - v[f, b]
            vals.append(oracle_lib.gather_e(sim, f, L, e) @ t)
        assert abs(vals[0] - vals[1]) <= 1e-12 * max(1.0, abs(vals[0]))
        # and the tangential integral along the edge equals the DoF itself
        assert abs(vals[0] - e[ed]) <= 1e-12 * max(1.0, abs(e[ed]))


def test_uniform_b_reproduced(oracle_lib):
    """b_f = Bz A_f gives Bz = b_f W2_f = b_f / A_f exactly; a uniform-B run
    with E = 0 never changes b (C e = 0)."""
    m = I.grid_mesh(9, 9, 1.0, 1.0)
    sim = _sim(oracle_lib, m)
    sim.b[:] = 0.37 * sim.T.area
    b0 = sim.b.copy()
    sim.step(3)
    assert np.all(sim.b == b0)
    assert np.allclose(sim.b / sim.T.area, 0.37, rtol=1e-15)


def test_curl_of_gradient_is_zero(oracle_lib):
    """Faraday update of an exact (gradient) e leaves b untouched."""
    m, T = _topo(oracle_lib, 10, 10, 1.0, 1.0)
    phi = np.random.default_rng(1).normal(size=T.nn)
    e = phi[T.edge_hi] - phi[T.edge_lo]
    sim = _sim(oracle_lib, m)
    out = np.empty(T.nf)
    import ctypes
    oracle_lib.lib().o_faraday(ctypes.byref(sim.ms), oracle_lib._p(sim.b), oracle_lib._p(e),
                               1.0, None, oracle_lib._p(out))
    assert np.abs(out).max() <= 1e-14 * np.abs(phi).max()


def test_hodge_eps_spd_and_quadrature(oracle_lib):
    """[*eps] is SPD (Sec. II.A) and each element contribution equals a
    degree-2 quadrature of eps0 W1_k . W1_l (edge-midpoint rule, exact for
    the quadratic integrand)."""
    m, T = _topo(oracle_lib, 9, 9, 1.0, 1.0)
    ptr, col, val = oracle_lib.hodge_eps(T, I.EPS0)
    M = oracle_lib.csr_to_dense(T.ne, ptr, col, val)
    assert np.allclose(M, M.T, rtol=0, atol=1e-14 * np.abs(M).max())
    free = T.edge_free.astype(bool)
    w = np.linalg.eigvalsh(M[np.ix_(free, free)])
    assert w.min() > 0
    G = T.grad.reshape(-1, 3, 2)
    # Element matrix against a degree-2 quadrature (edge-midpoint rule)
    rng = np.random.default_rng(2)
    for f in rng.integers(0, T.nf, 10):
        mids = [(np.array([0, .5, .5])), np.array([.5, 0, .5]), np.array([.5, .5, 0])]
        Wq = []
        for L in mids:
            Ws = []
            for k in range(3):
                a, b = (k + 1) % 3, (k + 2) % 3
                Ws.append(T.tri_sign[f, k] * (L[a] * G[f, b] - L[b] * G[f, a]))
            Wq.append(Ws)
        for k in range(3):
            for l in range(3):
                ek, el = T.tri_edge[f, k], T.tri_edge[f, l]
                quad = I.EPS0 * T.area[f] / 3 * sum(Wq[q][k] @ Wq[q][l] for q in range(3))
                # element contribution = assembled entry minus the other triangle's
                other = 0.0
                for j in range(2):
                    g = T.edge_tri[ek, j]
                    if g >= 0 and g != f and el in T.tri_edge[g]:
                        kk = int(np.nonzero(T.tri_edge[g] == ek)[0][0])
                        ll = int(np.nonzero(T.tri_edge[g] == el)[0][0])
                        Lm = [np.array([0, .5, .5]), np.array([.5, 0, .5]), np.array([.5, .5, 0])]
                        s = 0.0
                        for L in Lm:
                            def W(kq):
                                a, b = (kq + 1) % 3, (kq + 2) % 3
                                return T.tri_sign[g, kq] * (L[a] * G[g, b] - L[b] * G[g, a])
                            s += W(kk) @ W(ll)
                        other += I.EPS0 * T.area[g] / 3 * s
                if free[ek] and free[el]:
                    assert abs(M[ek, el] - (quad + other)) <= 1e-12 * abs(M[ek, ek])


def test_uniform_field_energy_periodic(oracle_lib):
    """On a torus every edge is free: e^T [*eps] e = eps0 |E|^2 * area."""
    m, T = _topo(oracle_lib, 8, 9, 0.5, 0.6, True, True)
    ptr, col, val = oracle_lib.hodge_eps(T, I.EPS0)
    start, dl = _edge_vec(T)
    E = np.array([2.0, -0.5])
    e = dl @ E
    en = e @ oracle_lib.csr_matvec(ptr, col, val, e)
    ref = I.EPS0 * (E @ E) * 0.5 * 0.6
    assert abs(en - ref) <= 1e-12 * ref


def test_spai_pins(oracle_lib):
    """Frobenius SPAI (Sec. II.A): the Frobenius residual ||I - M M~||_F
    falls with the pattern level (the paper's tunable accuracy); with a
    pattern covering the whole matrix it is the exact inverse; for a
    diagonal matrix level 0 is already exact."""
    m, T = _topo(oracle_lib, 6, 6, 1.0, 1.0, True, True)
    Me = oracle_lib.hodge_eps(T, I.EPS0)
    M = oracle_lib.csr_to_dense(T.ne, *Me)
    res = []
    for lvl in range(0, 4):
        Mt = oracle_lib.approx_inverse(T, Me, lvl)
        D = oracle_lib.csr_to_dense(T.ne, *Mt)
        assert np.allclose(D, D.T, rtol=0, atol=1e-12 * np.abs(D).max())
        res.append(np.linalg.norm(np.eye(T.ne) - M @ D))
    assert all(res[i + 1] < res[i] for i in range(len(res) - 1)), res
    assert res[-1] < 0.2 * res[0]
    # positive definite at the levels used for time stepping
    for lvl in (1, 2):
        D = oracle_lib.csr_to_dense(T.ne, *oracle_lib.approx_inverse(T, Me, lvl))
        assert np.linalg.eigvalsh(D).min() > 0
    # full pattern (tiny torus, large level) == exact inverse
    m2, T2 = _topo(oracle_lib, 3, 3, 1.0, 1.0, True, True)
    Me2 = oracle_lib.hodge_eps(T2, I.EPS0)
    M2 = oracle_lib.csr_to_dense(T2.ne, *Me2)
    D2 = oracle_lib.csr_to_dense(T2.ne, *oracle_lib.approx_inverse(T2, Me2, 6))
    assert np.abs(D2 - np.linalg.inv(M2)).max() <= 1e-9 * np.abs(np.linalg.inv(M2)).max()
    # diagonal matrix: level 0 is exact
    n = 5
    dptr = np.arange(n + 1, dtype=np.int32)
    dcol = np.arange(n, dtype=np.int32)
    dval = np.array([1.0, 2.0, 4.0, 0.5, 3.0])
    optr = np.zeros(n + 1, dtype=np.int32)
    ocol = np.zeros(n * 64, dtype=np.int32)
    oval = np.zeros(n * 64)
    nnz = oracle_lib.lib().o_spai(n, oracle_lib._p(dptr), oracle_lib._p(dcol),
                                  oracle_lib._p(dval), 0, oracle_lib._p(optr),
                                  oracle_lib._p(ocol), oracle_lib._p(oval), n * 64)
    assert nnz == n
    assert np.all(oval[:n] == 1.0 / dval)
