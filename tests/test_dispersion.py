"""The dispersion diagnostic (Sec. III.C): the textbook non-relativistic
Bernstein relation and the space-time spectrum.  Pins: roots are zeros of
eps_xx; the upper-hybrid limit omega^2 = omega_c^2 + sum omega_p^2 as
k -> 0 in its band (cold plasma); modes crowd to the harmonics at large k;
roots agree with a brute-force sign scan; a synthetic plane wave peaks at
its own (k, omega).

The relativistic relation (Sec. III.C eq. e_xx) is pinned by: the closed
form of G against the direct harmonic sum; the paper's integral
representation of 2F3 against its defining series; the principal value
and residues against the same average taken at a complex frequency
w + i nu (harmonic sum, no poles on the path) as nu -> 0; the long-
wavelength expansion against its own quadrature; the non-relativistic
limit (eta -> infinity) against the textbook relation, with the gap
shrinking as 1/eta; the three-dimensional average against the printed
2F3 form under the momentum integral."""
import math

import numpy as np
from scipy import integrate, special

from paper_1707_04333_amd import dispersion as D

VTH = np.sqrt(0.005)
WP2 = 0.5


def test_roots_are_zeros_of_eps_xx():
    k = np.array([1.0, 4.0, 9.0, 16.0, 25.0])
    m = D.bernstein_modes(k, VTH, WP2)
    for bi in range(m.shape[0]):
        for ki, kv in enumerate(k):
            w = m[bi, ki]
            # a simple zero: eps_xx changes sign across it (steep near a harmonic)
            lo = D.eps_xx(w - 1e-10, kv, VTH, WP2)
            hi = D.eps_xx(w + 1e-10, kv, VTH, WP2)
            assert lo * hi <= 0.0 and abs(D.eps_xx(w, kv, VTH, WP2)) < 1e-6


def test_upper_hybrid_limit():
    w = D.bernstein_modes([0.05], VTH, WP2, bands=(1,))[0, 0]
    assert abs(w - np.sqrt(1.0 + WP2)) < 1e-4


def test_modes_approach_harmonics_at_large_k():
    m = D.bernstein_modes([400.0], VTH, WP2, bands=(1, 2, 3))
    assert np.all(np.abs(m[:, 0] - np.array([1.0, 2.0, 3.0])) < 0.01)


def test_brute_force_sign_scan():
    k = 12.0
    grid = np.linspace(1.0 + 1e-6, 2.0 - 1e-6, 20001)
    vals = np.array([D.eps_xx(w, k, VTH, WP2) for w in grid])
    flips = np.nonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    assert flips.size == 1
    root = D.bernstein_modes([k], VTH, WP2, bands=(1,))[0, 0]
    assert grid[flips[0]] <= root <= grid[flips[0] + 1]


def test_spectrum_peaks_at_a_plane_wave():
    nx, nt, dx, dt = 128, 512, 1e-4, 2e-12
    omega_c, c = 1e11, 3e8
    j0, m0 = 9, 40
    x = np.arange(nx) * dx
    t = np.arange(nt) * dt
    k0 = 2 * np.pi * j0 / (nx * dx)
    w0 = 2 * np.pi * m0 / (nt * dt)
    ex = np.cos(k0 * x[None, :] - w0 * t[:, None])
    samples = np.stack([ex, np.zeros_like(ex)], axis=-1)
    k_hat, w, p = D.spectrum(samples, dt, dx, omega_c, c)
    wi, ki = np.unravel_index(np.argmax(p), p.shape)
    assert ki == j0 and wi == m0
    assert abs(k_hat[ki] - k0 * c / omega_c) < 1e-9 * k_hat[ki]
    assert abs(w[wi] - w0 / omega_c) < 1e-9 * w[wi]


# ---- relativistic relation (eq. e_xx) ----

def test_g_closed_form_matches_harmonic_sum():
    for a, z in ((0.3, 0.5), (1.37, 2.0), (2.61, 7.5), (5.2, 3.0), (0.97, 12.0)):
        r, s = D.g_parts(a, z)
        closed = r + s / math.tan(math.pi * a)
        assert abs(closed - D.g_newberger(a, z)) <= 1e-10 * max(1.0, abs(closed)), (a, z)
    assert D.g_parts(1.5, 0.0) == (1.0, 0.0)


def test_2f3_integral_representation_matches_series():
    for a, b in ((0.4, 0.8), (1.3, 2.0), (2.7, 4.0), (0.15, 6.0)):
        ser = D.hyp2f3_series(a, b)
        assert abs(D.hyp2f3_integral(a, b) - ser) <= 1e-10 * max(1.0, abs(ser)), (a, b)
        r3, s3 = D._polar_parts(a, b)
        assert abs(r3 + s3 / math.tan(math.pi * a) - ser) <= 1e-10 * max(1.0, abs(ser)), (a, b)


def _avg_g_complex(w, nu, k_hat, eta):
    """<G> over the 2-D Maxwell-Juttner distribution at the complex
    frequency w + i nu, from the harmonic sum (integer orders only)."""
    gmax = 1.0 + 45.0 / eta
    norm = eta * eta / (1.0 + eta)
    z_max = k_hat * math.sqrt(gmax * gmax - 1.0)
    n_max = int(z_max + 12.0 * z_max ** (1.0 / 3.0) + 30.0)
    wc = complex(w, nu)
    tot = 1.0 + 0.0j
    for n in range(1, n_max + 1):
        for sgn in (1, -1):
            m = sgn * n
            def f(g, part):
                p = math.sqrt(max(g * g - 1.0, 0.0))
                v = m * special.jv(n, k_hat * p) ** 2 / (g * wc - m) * g * math.exp(-eta * (g - 1.0))
                return v.real if part == 0 else v.imag
            pts = [m / w] if 1.0 < m / w < gmax else None
            for part in (0, 1):
                val = integrate.quad(f, 1.0, gmax, args=(part,), points=pts, limit=2000,
                                     epsabs=1e-15, epsrel=1e-12)[0]
                tot += norm * (val if part == 0 else 1j * val)
    return tot


def test_principal_value_is_the_limit_from_above():
    w, k_hat, eta = 1.5, 1.0, 10.0     # poles at gamma = 4/3, 2, 8/3, ...
    want = D.mj_average_g(w, k_hat, eta)
    g1 = _avg_g_complex(w, 4e-3, k_hat, eta)
    g2 = _avg_g_complex(w, 2e-3, k_hat, eta)
    lim = 2.0 * g2 - g1                 # the error is linear in nu
    assert abs(want.imag) > 1e-3
    assert abs(lim.real - want.real) <= 2e-4 * abs(want.real - 1.0), (lim, want)
    assert abs(lim.imag - want.imag) <= 1e-3 * abs(want.imag), (lim, want)


def test_long_wavelength_expansion():
    """k -> 0: G - 1 -> -z^2/(2(1 - a^2)), so eps_xx -> 1 + wp2 eta
    <p^2 / (2(1 - gamma^2 w^2))> over the 2-D distribution."""
    eta, wp2, k_hat = 10.0, 0.5, 1e-3
    for w in (1.3, 2.4):
        num = integrate.quad(lambda g: (g * g - 1.0) / (2.0 * (1.0 - g * g * w * w)) * g *
                             math.exp(-eta * (g - 1.0)), 1.0, 1.0 + 45.0 / eta,
                             epsabs=1e-15, epsrel=1e-12)[0]
        want = 1.0 + wp2 * eta * num * eta * eta / (1.0 + eta)
        got = D.eps_xx_rel(w, k_hat, eta, wp2)
        assert abs(got.real - want) <= 1e-5 * abs(want), (w, got, want)


def test_nonrelativistic_limit():
    wp2 = 0.5
    for w, k_hat in ((0.5, 0.2), (1.5, 2.0), (2.5, 5.0)):
        gaps = []
        for eta in (2000.0, 4000.0):
            rel = D.eps_xx_rel(w, k_hat, eta, wp2).real
            cl = D.eps_xx(w, k_hat, math.sqrt(1.0 / eta), wp2)
            gaps.append(abs(rel - cl))
            assert gaps[-1] <= 20.0 / eta * max(1.0, abs(cl)), (w, k_hat, eta, rel, cl)
        assert 1.6 < gaps[0] / gaps[1] < 2.4, gaps


def test_three_dimensional_average_is_the_printed_form():
    """Where no resonance lies in the momentum range (w = 0.05 at eta = 10)
    the 3-D average equals eq. e_xx's integral of p^2 exp(-eta gamma) 2F3
    over p, normalised by K_2(eta)/eta."""
    w, k_hat, eta = 0.05, 3.0, 10.0
    got = D.mj_average_g(w, k_hat, eta, dim=3)
    assert got.imag == 0.0

    def f(p):
        g = math.sqrt(1.0 + p * p)
        return p * p * math.exp(-eta * (g - 1.0)) * D.hyp2f3_series(g * w, k_hat * p)
    pmax = math.sqrt((1.0 + 45.0 / eta) ** 2 - 1.0)
    want = eta / special.kve(2, eta) * integrate.quad(f, 0.0, pmax, epsabs=1e-15, epsrel=1e-12)[0]
    assert abs(got.real - want) <= 1e-9 * abs(want), (got, want)


def test_relativistic_roots_are_zeros():
    for k_hat in (0.3, 1.5):
        modes = D.rel_bernstein_modes(k_hat, 10.0, 0.5, 1)
        assert modes
        for w, damp in modes:
            assert abs(D.eps_xx_rel(w, k_hat, 10.0, 0.5).real) < 1e-7
