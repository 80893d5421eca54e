"""Pins of the oracle pushers against what the paper and the mathematics fix.

Each pusher is defined in Sec. II.C by its averaged velocity v-bar in the
central-difference momentum equation (eq. Lorentz.Newton.dis):
    u^{n+1/2} - u^{n-1/2} = 2 eps + dt (q/m) v-bar x B  =  2 eps + 2 v-bar x beta
  Boris  : v-bar = (u+ + u-) / (2 gamma(u-)),  u- = u + eps, u+ = u_new - eps
           with gamma(u-) = gamma(u+)                       (eq. gamma.middle)
  Vay    : v-bar = (v(u^{n+1/2}) + v(u^{n-1/2})) / 2
  HC     : v-bar = v((u^{n+1/2} + u^{n-1/2}) / 2)
These implicit equations are checked on the oracle's explicit updates, so a
dropped term, a wrong sign or a swapped operand in the update fails here.
"""
import math

import numpy as np
import pytest

C = 299792458.0


def vel(u):
    return u / math.sqrt(1.0 + u @ u / C ** 2)


def rand_case(rng, umax=3.0, emax=0.3, bmax=0.5):
    u = rng.normal(size=3) * C * umax
    eps = rng.normal(size=3) * C * emax
    beta = rng.normal(size=3) * bmax
    return u, eps, beta


@pytest.mark.parametrize("seed", range(20))
def test_boris_implicit_equation(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    u, eps, beta = rand_case(rng)
    out = oracle_lib.push_raw("boris", u, eps, beta, C)
    um, up = u + eps, out - eps
    g = math.sqrt(1 + um @ um / C ** 2)
    lhs = up - um
    rhs = np.cross(up + um, beta) / g
    assert np.abs(lhs - rhs).max() <= 1e-14 * np.abs(um).max()
    # |u+| = |u-|: the magnetic rotation conserves gamma (eq. gamma.middle)
    assert abs(np.linalg.norm(up) - np.linalg.norm(um)) <= 1e-14 * np.linalg.norm(um)


@pytest.mark.parametrize("seed", range(20))
def test_vay_implicit_equation(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    u, eps, beta = rand_case(rng)
    out = oracle_lib.push_raw("vay", u, eps, beta, C)
    lhs = out - u
    rhs = 2 * eps + np.cross(vel(out) + vel(u), beta)
    assert np.abs(lhs - rhs).max() <= 2e-14 * max(np.abs(u).max(), np.abs(out).max())


@pytest.mark.parametrize("seed", range(20))
def test_hc_implicit_equation(oracle_lib, seed):
    rng = np.random.default_rng(200 + seed)
    u, eps, beta = rand_case(rng)
    out = oracle_lib.push_raw("hc", u, eps, beta, C)
    lhs = out - u
    rhs = 2 * eps + 2 * np.cross(vel(0.5 * (out + u)), beta)
    assert np.abs(lhs - rhs).max() <= 2e-14 * max(np.abs(u).max(), np.abs(out).max())


@pytest.mark.parametrize("seed", range(10))
def test_boris_tan_is_exact_rotation(oracle_lib, seed):
    """With the tan correction the magnetic rotation of u- about beta is by
    exactly 2|beta|/gamma-bar (Sec. II.C(a))."""
    rng = np.random.default_rng(300 + seed)
    u, eps, beta = rand_case(rng)
    out = oracle_lib.push_raw("boris_tan", u, eps, beta, C)
    um, up = u + eps, out - eps
    g = math.sqrt(1 + um @ um / C ** 2)
    bm = np.linalg.norm(beta)
    n = beta / bm
    th = -2 * bm / g  # u' = u- + u- x t rotates u- about -n (v x B force sense)
    rot = (um * math.cos(th) + np.cross(n, um) * math.sin(th)
           + n * (n @ um) * (1 - math.cos(th)))
    assert np.abs(up - rot).max() <= 1e-13 * np.abs(um).max()


@pytest.mark.parametrize("pusher", ["boris", "boris_tan", "vay", "hc"])
def test_pure_electric_kick(oracle_lib, pusher):
    """B = 0: every pusher gives u^{n+1/2} = u^{n-1/2} + 2 eps."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        u, eps, _ = rand_case(rng)
        out = oracle_lib.push_raw(pusher, u, eps, np.zeros(3), C)
        assert np.abs(out - (u + 2 * eps)).max() <= 1e-15 * np.abs(u + 2 * eps).max()


@pytest.mark.parametrize("pusher,exact", [("vay", True), ("hc", True), ("boris", False)])
@pytest.mark.parametrize("vd", [0.866, 0.98, 0.995])
def test_exb_drift(oracle_lib, pusher, exact, vd):
    """Pure E x B drift (E + v x B = 0): Vay and Higuera-Cary keep the
    drifting particle's momentum unchanged; Boris does not (the paper's
    comparison in Sec. III.B)."""
    bmag = 0.1
    beta = np.array([0.0, 0.0, bmag])
    v = np.array([vd * C, 0.0, 0.0])
    g = 1 / math.sqrt(1 - vd ** 2)
    u = g * v
    eps = -np.cross(v, beta)  # alpha E = -alpha v x B
    out = oracle_lib.push_raw(pusher, u, eps, beta, C)
    err = np.abs(out - u).max() / C
    if exact:
        assert err < 1e-14
    else:
        assert err > 1e-6


def _hc_angle(u, bm):
    """Rotation half-angle T = tan(theta/2) of Higuera-Cary for E = 0,
    derived from its implicit definition: v-bar = v(u-bar) with u-bar the
    chord midpoint, |u-bar| = |u| cos(theta/2), gives gamma_H^2 =
    1 + u^2 / (c^2 (1 + T^2)) and T = |beta| / gamma_H."""
    u2 = u * u / C ** 2
    # gamma_H^2 = 1 + u2 gamma_H^2 / (gamma_H^2 + bm^2)  ->  G^2 - (1+u2-b^2) G - b^2 = 0
    bb = bm * bm
    G = 0.5 * ((1 + u2 - bb) + math.sqrt((1 + u2 - bb) ** 2 + 4 * bb))
    return bm / math.sqrt(G)


@pytest.mark.parametrize("pusher", ["boris", "boris_tan", "vay", "hc"])
def test_gyration_angle(oracle_lib, pusher):
    """E = 0, uniform B: |u| is conserved and the per-step rotation angle
    theta is tan(theta/2) = |beta|/gamma (Boris, Vay), 2|beta|/gamma
    (Boris with tan correction) or tan(theta/2) = |beta|/gamma_H (HC)."""
    for gam in [1.0 + 1e-6, 1.5, 3.0, 10.0]:
        um = C * math.sqrt(gam * gam - 1)
        u = np.array([um, 0.0, 0.0])
        for bm in [1e-3, 0.1, 0.7]:
            out = oracle_lib.push_raw(pusher, u, np.zeros(3), np.array([0, 0, bm]), C)
            assert abs(np.linalg.norm(out) - um) <= 2e-15 * um
            th = math.atan2(-out[1], out[0])  # positive beta rotates clockwise
            if pusher in ("boris", "vay"):
                ref = 2 * math.atan(bm / gam)
            elif pusher == "boris_tan":
                ref = 2 * bm / gam
            else:
                ref = 2 * math.atan(_hc_angle(um, bm))
            assert abs(th - ref) <= 1e-13 * max(1.0, abs(ref))


def test_nonrelativistic_limit(oracle_lib):
    """c -> infinity: the relativistic Boris map tends to the classical
    Boris rotation, an exact rotation by 2 atan(|beta|) (Sec. II.C)."""
    big_c = 1e30
    u = np.array([1.0e6, 2.0e5, 0.0])
    bm = 0.3
    out = oracle_lib.push_raw("boris", u, np.zeros(3), np.array([0, 0, bm]), big_c)
    th = 2 * math.atan(bm)
    rot = np.array([u[0] * math.cos(th) + u[1] * math.sin(th),
                    -u[0] * math.sin(th) + u[1] * math.cos(th), 0.0])
    assert np.abs(out - rot).max() <= 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("pusher,preserving", [("boris", True), ("hc", True),
                                               ("boris_tan", True), ("vay", False)])
def test_phase_space_volume(oracle_lib, pusher, preserving):
    """det d u^{n+1/2} / d u^{n-1/2} = 1 for Boris and Higuera-Cary with
    fields fixed over the step (Sec. II.C, eq. eq.Jacob and below);
    the Vay map is not volume preserving."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(5):
        u, eps, beta = rand_case(rng, umax=2.0, emax=0.2, bmax=0.6)
        J = np.zeros((3, 3))
        h = 1e-4 * C
        for j in range(3):
            du = np.zeros(3)
            du[j] = h
            fp = oracle_lib.push_raw(pusher, u + du, eps, beta, C)
            fm = oracle_lib.push_raw(pusher, u - du, eps, beta, C)
            J[:, j] = (fp - fm) / (2 * h)
        worst = max(worst, abs(np.linalg.det(J) - 1.0))
    if preserving:
        assert worst < 1e-7
    else:
        assert worst > 1e-4
