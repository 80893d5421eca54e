"""Pins of the oracle's particle tracking against exact rational geometry.

The exact current of eq. I.assign (Sec. II.D) holds for a straight path
inside one triangle, so a move must be split at every triangle edge it
crosses.  The brute force here clips the straight path against every
triangle of a tiny mesh in exact rational arithmetic (Python fractions)
and yields the sequence of triangles the path runs through with positive
length and the parameter at which it enters each; the oracle must report
the same sequence and the same split points (to rounding).  Zero-length
pieces (vertex passes) carry no current and are not compared."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I


def _mesh(periodic):
    if periodic:
        return I.grid_mesh(6, 5, 1.0, 0.8, True, True, seed=5)
    return I.grid_mesh(7, 6, 1.0, 0.9, seed=5)


def _sim(oracle_lib, m):
    return oracle_lib.OracleSim(m, 1e-12, [], I.EPS0, I.MU0, I.C_LIGHT, spai_level=1)


def _image_triangles(sim, m):
    """Triangles as exact rational vertex lists, with periodic images."""
    v = sim.T.vxy.reshape(-1, 3, 2)
    out = []
    shifts = [(0, 0)]
    if m.period is not None:
        px, py = m.period
        shifts = [(sx * px, sy * py) for sx in ((-1, 0, 1) if px else (0,))
                  for sy in ((-1, 0, 1) if py else (0,))]
    for f in range(sim.T.nf):
        for sx, sy in shifts:
            out.append((f, [(Fr(v[f, k, 0]) + Fr(sx), Fr(v[f, k, 1]) + Fr(sy))
                            for k in range(3)]))
    return out


def _clip(tris, P, D):
    """Exact pieces of P + t D, t in [0,1], per triangle: (t_in, t_out, f)."""
    pieces = []
    x0, x1 = sorted([float(P[0]), float(P[0] + D[0])])
    y0, y1 = sorted([float(P[1]), float(P[1] + D[1])])
    for f, V in tris:
        vx = [float(p[0]) for p in V]
        vy = [float(p[1]) for p in V]
        if max(vx) < x0 - 1e-9 or min(vx) > x1 + 1e-9 or max(vy) < y0 - 1e-9 or min(vy) > y1 + 1e-9:
            continue
        lo, hi = Fr(0), Fr(1)
        ok = True
        for k in range(3):
            A, B = V[(k + 1) % 3], V[(k + 2) % 3]
            # signed area of (A, B, X) >= 0 inside a CCW triangle
            def s(t):
                X = (P[0] + t * D[0], P[1] + t * D[1])
                return (B[0] - A[0]) * (X[1] - A[1]) - (B[1] - A[1]) * (X[0] - A[0])
            s0, s1 = s(Fr(0)), s(Fr(1))
            ds = s1 - s0
            if ds == 0:
                if s0 < 0:
                    ok = False
                    break
                continue
            tz = -s0 / ds
            if ds > 0:
                lo = max(lo, tz)
            else:
                hi = min(hi, tz)
        if ok and hi > lo:
            pieces.append((lo, hi, f))
    pieces.sort()
    return pieces


def _start(rng, sim, f):
    """A start point with exactly representable barycentrics."""
    lam = rng.dirichlet([1, 1, 1])
    pair = np.array([lam[1], lam[2]])
    L0 = (1.0 - pair[0]) - pair[1]
    v = sim.T.vxy.reshape(-1, 3, 2)[f]
    P = tuple(Fr(L0) * Fr(v[0, i]) + Fr(pair[0]) * Fr(v[1, i]) + Fr(pair[1]) * Fr(v[2, i])
              for i in range(2))
    return pair, P


@pytest.mark.parametrize("periodic", [False, True])
def test_crossing_sequence_matches_exact_clipping(oracle_lib, periodic):
    m = _mesh(periodic)
    sim = _sim(oracle_lib, m)
    tris = _image_triangles(sim, m)
    rng = np.random.default_rng(17 if periodic else 18)
    h = 1.0 / 6
    checked = crossings = 0
    for trial in range(120):
        f0 = int(rng.integers(sim.T.nf))
        pair, P = _start(rng, sim, f0)
        ang = rng.uniform(0, 2 * np.pi)
        dist = rng.uniform(0.05, 3.0) * h
        D = (float(dist * np.cos(ang)), float(dist * np.sin(ang)))
        Dq = (Fr(D[0]), Fr(D[1]))
        pieces = _clip(tris, P, Dq)
        # the exact path starts in f0 (the start is inside f0)
        t_end = pieces[-1][1] if pieces else Fr(0)
        ft, fs, fpair, lost, segs, cur = oracle_lib.move_one(sim, f0, 0, pair, D[0], D[1])
        segs = [s for s in segs if not np.array_equal(s[1], s[2])]
        # merge exact pieces of the same triangle that are contiguous
        exact = []
        for lo, hi, f in pieces:
            if hi - lo <= Fr(1, 10 ** 12):
                continue
            exact.append((f, lo, hi))
        if any(hi - lo < Fr(1, 10 ** 9) for _, lo, hi in exact):
            continue  # near-degenerate grazing case; covered by validity tests
        assert [s[0] for s in segs] == [f for f, _, _ in exact], trial
        # split points agree with the exact entry parameters
        v = sim.T.vxy.reshape(-1, 3, 2)
        for (f, lo, hi), s in zip(exact, segs):
            xe = np.array([float(P[0] + hi * Dq[0]), float(P[1] + hi * Dq[1])])
            xo = s[2] @ v[f]
            if m.period is not None:
                d = xe - xo
                d -= np.round(d / m.period) * m.period
                assert np.abs(d).max() < 1e-12
            else:
                assert np.abs(xe - xo).max() < 1e-12
        assert lost == (t_end < 1)
        checked += 1
        crossings += len(segs) - 1
    assert checked > 100 and crossings > 50


def test_edge_cases(oracle_lib):
    m = _mesh(False)
    sim = _sim(oracle_lib, m)
    T = sim.T
    v = T.vxy.reshape(-1, 3, 2)
    f = int(np.nonzero(np.all(T.tri_nbr >= 0, axis=1))[0][0])
    # zero move: one segment, unchanged position, no current
    ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, f, 0, [0.2, 0.3], 0.0, 0.0)
    assert ft == f and fs == 0 and list(pr) == [0.2, 0.3] and len(segs) == 1
    assert not np.any(cur) and not lost
    # start on local edge 0 (lambda_0 = 0) moving out through it: an
    # immediate crossing into the neighbour with a zero-length piece
    g = v[f, 0]
    mid = 0.5 * (v[f, 1] + v[f, 2])
    out = (mid - g) * 0.3
    ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, f, 0, [0.5, 0.5], out[0], out[1])
    assert segs[0][0] == f and np.array_equal(segs[0][1], segs[0][2])
    assert ft != f and segs[1][0] == T.tri_nbr[f, 0]
    # the same start moving inward stays in f
    ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, f, 0, [0.5, 0.5], -out[0] * 0.1,
                                                      -out[1] * 0.1)
    assert ft == f and len(segs) == 1
    # start at a vertex: several continuations are geometrically valid;
    # the result must be a valid interior point of its final triangle
    rng = np.random.default_rng(3)
    for _ in range(30):
        ang = rng.uniform(0, 2 * np.pi)
        d = 0.02 * np.array([np.cos(ang), np.sin(ang)])
        ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, f, 0, [0.0, 0.0], d[0], d[1])
        if lost:
            continue
        L = np.zeros(3)
        L[(fs + 1) % 3], L[(fs + 2) % 3] = pr
        L[fs] = (1 - pr[0]) - pr[1]
        assert L.min() > -1e-12
        x = L @ v[ft]
        assert np.abs(x - (v[f, 0] + d)).max() < 1e-12
    # crossing cap: a long move with cap 1 is an error
    with pytest.raises(RuntimeError):
        oracle_lib.move_one(sim, f, 0, [0.3, 0.3], 0.5, 0.1, cap=1)


def test_wall_loss(oracle_lib):
    """A path that meets the PEC wall ends there and the particle is lost
    (Sec. III: walls absorb; only free DoFs are evolved)."""
    m = _mesh(False)
    sim = _sim(oracle_lib, m)
    T = sim.T
    bnd = np.nonzero(np.any(T.tri_nbr < 0, axis=1))[0]
    rng = np.random.default_rng(9)
    n_lost = 0
    for f in bnd[:20]:
        k = int(np.nonzero(T.tri_nbr[f] < 0)[0][0])
        v = T.vxy.reshape(-1, 3, 2)[f]
        a, b = (k + 1) % 3, (k + 2) % 3
        mid = 0.5 * (v[a] + v[b])
        d = (mid - v[k]) * 2.0
        ft, fs, pr, lost, segs, cur = oracle_lib.move_one(sim, int(f), 0, [1 / 3, 1 / 3],
                                                          d[0], d[1])
        assert lost
        n_lost += 1
        # last piece ends on the wall edge (its opposite barycentric is 0)
        last_f, Ls, Lf = segs[-1]
        assert np.min(np.abs(Lf)) == 0.0
    assert n_lost == 20


def test_step_records_each_particles_pieces(oracle_lib):
    """The oracle's per-particle piece record of a step (the triangle of each
    straight piece, Sec. II.D): it starts in the particle's triangle before
    the step, walks through edge neighbours, ends in its triangle after the
    step (unless lost at a wall), and the piece counts sum to the step's
    segment count."""
    w = I.pair_plasma(n_side=12, length=0.02, n_pairs=1500, theta=1.0, steps=5,
                      precision="fp64")
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = oracle_lib.OracleSim(w.mesh, w.dt * 3.0, sp, I.EPS0, I.MU0, I.C_LIGHT,
                                spai_level=1, bz_ext=w.bz_ext)
    T = osim.T
    K = 6
    crossed = 0
    for _ in range(4):
        before = [s.tri.copy() for s in osim.species]
        seg0 = osim.segments
        osim.step(1, "hc", record=K)
        total = 0
        for s, b in zip(osim.species, before):
            alive = b >= 0
            assert np.all(s.nseq[~alive] == 0)
            assert np.all(s.nseq[alive] >= 1)
            assert np.array_equal(s.seq[alive, 0], b[alive])
            total += int(s.nseq.sum())
            for p in np.nonzero(alive)[0]:
                m = min(int(s.nseq[p]), K)
                for k in range(1, m):
                    assert s.seq[p, k] in T.tri_nbr[s.seq[p, k - 1]]
                assert np.all(s.seq[p, m:] == -1)
                if s.nseq[p] <= K and s.tri[p] >= 0:
                    assert s.seq[p, m - 1] == s.tri[p]
            crossed += int((s.nseq[alive] > 1).sum())
        assert total == osim.segments - seg0
    assert crossed > 1000
