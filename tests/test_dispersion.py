"""The dispersion diagnostic (Sec. III.C): the textbook non-relativistic
Bernstein relation and the space-time spectrum.  Pins: roots are zeros of
eps_xx; the upper-hybrid limit omega^2 = omega_c^2 + sum omega_p^2 as
k -> 0 in its band (cold plasma); modes crowd to the harmonics at large k;
roots agree with a brute-force sign scan; a synthetic plane wave peaks at
its own (k, omega)."""
import numpy as np

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
