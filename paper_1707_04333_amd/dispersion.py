"""Dispersion diagnostic of Sec. III.C: space-time Fourier transform of a
field probe line, and the non-relativistic (textbook) electrostatic
Bernstein dispersion relation it is compared with.

Bernstein waves propagate normal to B0 (here along x); for a Maxwellian of
thermal speed v_th (v_th^2 = k_B T / m) the longitudinal dielectric
function of species s is

    eps_xx / eps0 = 1 - sum_s (omega_ps/omega_c)^2 (2/lambda)
                          sum_{n>=1} n^2 e^-lambda I_n(lambda) / (w^2 - n^2),

lambda = (k v_th / omega_c)^2, w = omega/omega_c; the modes are its zeros,
one in each band n < w < n + 1 (the band holding the upper-hybrid
frequency starts from it as k -> 0).  For the pair plasma of Sec. III.C
both species have the same |q|/m, so the sum over species adds their
plasma frequencies squared.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize, special


def eps_xx(w: float, k_hat: float, vth_over_c: float, wp2_total: float, n_max: int = 0) -> float:
    """eps_xx/eps0 at normalised frequency w = omega/omega_c and wavenumber
    k_hat = k c/omega_c; wp2_total = sum_s (omega_ps/omega_c)^2."""
    lam = (k_hat * vth_over_c) ** 2
    if n_max <= 0:
        n_max = int(lam + 10.0 * np.sqrt(lam + 1.0) + 10.0 + w)
    n = np.arange(1, n_max + 1, dtype=np.float64)
    terms = n * n * special.ive(n, lam) / (w * w - n * n)
    return 1.0 - wp2_total * (2.0 / lam) * float(terms.sum())


def bernstein_modes(k_hat, vth_over_c: float, wp2_total: float, bands=(1, 2, 3)):
    """Mode frequency w(k) in each band (n, n+1) for the wavenumbers k_hat:
    array [len(bands), len(k_hat)] (NaN where no root is bracketed)."""
    k_hat = np.atleast_1d(np.asarray(k_hat, dtype=np.float64))
    out = np.full((len(bands), k_hat.size), np.nan)
    for bi, nb in enumerate(bands):
        for ki, k in enumerate(k_hat):
            lo, hi = nb + 1e-9, nb + 1 - 1e-9
            f = lambda w: eps_xx(w, k, vth_over_c, wp2_total)
            if f(lo) * f(hi) < 0:
                out[bi, ki] = optimize.brentq(f, lo, hi, xtol=1e-12)
    return out


def spectrum(samples: np.ndarray, dt_sample: float, dx: float, omega_c: float, c: float):
    """|E_x(k, omega)|^2 of probe samples [T, N, 2] taken on a uniform line
    along x (periodic in x, spacing dx) every dt_sample seconds, after
    removing each point's mean and applying a Hann window in time.  Waves
    travelling either way are summed: P(k, w) + P(-k, w).  Returns
    (k_hat [N//2+1], w [T//2+1], power [T//2+1, N//2+1]) with
    k_hat = k c/omega_c and w = omega/omega_c."""
    ex = np.asarray(samples[:, :, 0], dtype=np.float64)
    ex = ex - ex.mean(axis=0, keepdims=True)
    nt, nx = ex.shape
    F = np.fft.fft2(ex * np.hanning(nt)[:, None])
    P = np.abs(F) ** 2
    jpos = np.arange(nx // 2 + 1)
    jneg = (-jpos) % nx
    wpos = np.arange(nt // 2 + 1)
    power = P[np.ix_(wpos, jpos)] + P[np.ix_(wpos, jneg)]
    k_hat = 2.0 * np.pi * jpos / (nx * dx) * c / omega_c
    w = 2.0 * np.pi * wpos / (nt * dt_sample) / omega_c
    return k_hat, w, power


def ridge(k_hat, w, power, band):
    """Frequency of the strongest response in the open band (n, n+1) for each
    wavenumber column: array [len(k_hat)]."""
    n = band
    sel = (w > n + 0.02) & (w < n + 0.98)
    idx = np.argmax(power[sel, :], axis=0)
    return w[sel][idx]
