"""Dispersion diagnostic of Sec. III.C: space-time Fourier transform of a
field probe line, and the electrostatic Bernstein dispersion relations it
is compared with.

Bernstein waves propagate normal to B0 (here along x).  Non-relativistic
(textbook) form: for a Maxwellian of thermal speed v_th (v_th^2 = k_B T /
m) the longitudinal dielectric function is

    eps_xx / eps0 = 1 - sum_s (omega_ps/omega_c)^2 (2/lambda)
                          sum_{n>=1} n^2 e^-lambda I_n(lambda) / (w^2 - n^2),

lambda = (k v_th / omega_c)^2, w = omega/omega_c; the modes are its zeros,
one in each band n < w < n + 1 (the band holding the upper-hybrid
frequency starts from it as k -> 0).  For the pair plasma of Sec. III.C
both species have the same |q|/m, so the sum over species adds their
plasma frequencies squared.

Relativistic form (the Maxwell-Juttner plasma of Sec. III.C, eq. e_xx):
a particle of Lorentz factor gamma gyrates at omega_c/gamma, so with
a = gamma w, z = k_hat p_hat (p_hat = p/(m c), k_hat = k c/omega_c) the
orbit sum over harmonics collapses to

    G(a, z) = 1 + sum_n n J_n(z)^2 / (a - n)
            = (pi a / sin(pi a)) J_a(z) J_-a(z),

and for an isotropic equilibrium f0 ~ exp(-eta gamma) (eta = m c^2/k_B T)

    eps_xx / eps0 = 1 - (sum_s (omega_ps/omega_c)^2) (eta / k_hat^2) (<G> - 1),

<.> the average over f0.  The paper's equation averages over a
three-dimensional momentum distribution, where the polar-angle average
of G is the 2F3 function it prints; the simulated particles carry in-plane
momenta only, so the comparison with a run uses the same relation averaged
over the two-dimensional Maxwell-Juttner distribution (weight
gamma exp(-eta gamma) d gamma).  G has poles where a gamma-shell gyrates at
a harmonic of the wave (gamma = m/w); the real part here is their
principal value and the imaginary part their residues (the omega + i0
prescription), i.e. the weak-damping reading of the dispersion relation.
"""
from __future__ import annotations

import numpy as np
import math

from scipy import integrate, optimize, special


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


# ---------------------------------------------------------------------
# Relativistic (Maxwell-Juttner) Bernstein relation, Sec. III.C eq. e_xx.
# ---------------------------------------------------------------------
_TAIL = 45.0          # the gamma integral stops where exp(-eta (gamma-1)) < e^-45
_THETA_NODES = 48     # Gauss-Legendre nodes of the polar average (3-D form)


def g_newberger(a: float, z: float, n_max: int = 0) -> float:
    """G(a, z) = 1 + sum_{n != 0} n J_n(z)^2 / (a - n) by direct summation of
    the harmonic series (a not an integer)."""
    if n_max <= 0:
        n_max = int(abs(z) + 12.0 * abs(z) ** (1.0 / 3.0) + 40.0)
    n = np.arange(1, n_max + 1, dtype=np.float64)
    j2 = special.jv(n, z) ** 2
    return 1.0 + float(np.sum(n * j2 / (a - n) - n * j2 / (a + n)))


def g_parts(a: float, z: float):
    """The two parts of G(a, z) = (pi a/sin(pi a)) J_a(z) J_-a(z): with
    J_-a = cos(pi a) J_a - sin(pi a) Y_a, G = R + cot(pi a) S where
    R = -pi a J_a(z) Y_a(z) is regular in a and S = pi a J_a(z)^2 >= 0.
    G(a, 0) = 1 (R -> 1, S -> 0)."""
    if z == 0.0:
        return 1.0, 0.0
    ja = special.jv(a, z)
    return -math.pi * a * ja * special.yv(a, z), math.pi * a * ja * ja


def hyp2f3_series(a: float, b: float, tol: float = 1e-17) -> float:
    """2F3(1/2, 1; 3/2, 1-a, 1+a; -b^2) summed from its defining series."""
    term, total, n = 1.0, 1.0, 0
    x = -b * b
    while True:
        term *= (0.5 + n) * x / ((1.5 + n) * (1.0 - a + n) * (1.0 + a + n))
        n += 1
        total += term
        if abs(term) < tol * abs(total) and n > 2 + 2 * abs(b):
            return total
        if n > 100000:
            raise RuntimeError("2F3 series did not converge")


def hyp2f3_integral(a: float, b: float) -> float:
    """The integral representation printed beside eq. e_xx: one half of the
    integral over theta of (pi a/sin(pi a)) sin(theta) J_a(b sin theta)
    J_-a(b sin theta).  The printed upper limit is read as pi (the
    integrand is periodic in theta, so no other limit gives a finite
    value); the half-integral over [0, pi] equals the integral over
    [0, pi/2], the polar average over a hemisphere."""
    f = lambda t: (math.pi * a / math.sin(math.pi * a)) * math.sin(t) * \
        special.jv(a, b * math.sin(t)) * special.jv(-a, b * math.sin(t))
    return 0.5 * integrate.quad(f, 0.0, math.pi, limit=200, epsabs=1e-14, epsrel=1e-12)[0]


def _polar_parts(a: float, z: float):
    """Hemisphere averages of R and S (the two parts of G) at z sin(theta):
    the 2F3 of eq. e_xx is R3 + cot(pi a) S3."""
    x, wq = np.polynomial.legendre.leggauss(_THETA_NODES)
    t = 0.25 * math.pi * (x + 1.0)
    st = np.sin(t)
    zz = z * st
    ja = special.jv(a, zz)
    ya = special.yv(a, zz)
    wt = 0.25 * math.pi * wq * st
    return float(np.sum(wt * (-math.pi * a * ja * ya))), float(np.sum(wt * (math.pi * a * ja * ja)))


def _mj_weight(eta: float, dim: int):
    """Weight in gamma of the isotropic Maxwell-Juttner distribution (up to
    exp(-eta)) and its normalisation: 2-D, d^2p ~ gamma d gamma; 3-D,
    d^3p ~ p gamma d gamma (normalised by K_2(eta), as in eq. e_xx)."""
    if dim == 2:
        return (lambda g: g * math.exp(-eta * (g - 1.0))), eta * eta / (1.0 + eta)
    if dim == 3:
        return (lambda g: g * math.sqrt(max(g * g - 1.0, 0.0)) * math.exp(-eta * (g - 1.0))), \
            eta / special.kve(2, eta)
    raise ValueError("dim must be 2 or 3")


def mj_average_g(w: float, k_hat: float, eta: float, dim: int = 2) -> complex:
    """<G>(w + i0) over the Maxwell-Juttner distribution of temperature
    1/eta: principal value of the poles gamma_m = m/w (m > w) as the real
    part, minus i/w times the sum of the weighted residues as the imaginary
    part.  w must not be an integer."""
    weight, norm = _mj_weight(eta, dim)
    gmax = 1.0 + _TAIL / eta

    def parts(g):
        z = k_hat * math.sqrt(max(g * g - 1.0, 0.0))
        a = g * w
        r, s = g_parts(a, z) if dim == 2 else _polar_parts(a, z)
        return weight(g) * r, weight(g) * s

    opts = dict(limit=400, epsabs=1e-14, epsrel=1e-11)
    re = integrate.quad(lambda g: parts(g)[0], 1.0, gmax, **opts)[0]
    poles = [m / w for m in range(int(math.floor(w)) + 1, int(math.ceil(gmax * w)) + 1)
             if m / w < gmax]
    im = 0.0
    if not poles:
        re += integrate.quad(lambda g: parts(g)[1] / math.tan(math.pi * g * w), 1.0, gmax, **opts)[0]
    else:
        cuts = [1.0] + [0.5 * (poles[i] + poles[i + 1]) for i in range(len(poles) - 1)] + [gmax]
        for i, gm in enumerate(poles):
            # cot(pi g w) = [(g - gm) cot(pi g w)] / (g - gm): the bracket is
            # smooth at the pole, where it equals 1/(pi w).
            def smooth(g, gm=gm):
                x = g - gm
                c = 1.0 / (math.pi * w) if abs(x) < 1e-13 * gm else x / math.tan(math.pi * g * w)
                return parts(g)[1] * c
            re += integrate.quad(smooth, cuts[i], cuts[i + 1], weight="cauchy", wvar=gm, **opts)[0]
            im += parts(gm)[1] / w
    return complex(norm * re, -norm * im)


def eps_xx_rel(w: float, k_hat: float, eta: float, wp2_total: float, dim: int = 2) -> complex:
    """eps_xx/eps0 of the relativistic pair plasma (eq. e_xx) at w = omega /
    omega_c, k_hat = k c/omega_c, eta = m c^2/(k_B T), wp2_total = sum_s
    (omega_ps/omega_c)^2 (rest-mass plasma frequencies): real part the
    principal value, imaginary part the resonant (damping) part."""
    g = mj_average_g(w, k_hat, eta, dim)
    return 1.0 - wp2_total * eta / (k_hat * k_hat) * (g - 1.0)


def rel_bernstein_modes(k_hat: float, eta: float, wp2_total: float, band: int, dim: int = 2,
                        n_scan: int = 80):
    """Zeros of Re eps_xx in the open band (band, band+1) at one wavenumber:
    list of (w, damping) with damping = Im eps / (d Re eps / dw), the decay
    rate in units of omega_c of a weakly damped mode (large values mark a
    zero of the real part that is no mode)."""
    lo, hi = band + 1e-4, band + 1.0 - 1e-4
    grid = np.linspace(lo, hi, n_scan)
    f = lambda x: eps_xx_rel(x, k_hat, eta, wp2_total, dim).real
    vals = np.array([f(x) for x in grid])
    out = []
    for i in range(n_scan - 1):
        if vals[i] * vals[i + 1] < 0.0:
            r = optimize.brentq(f, grid[i], grid[i + 1], xtol=1e-10)
            h = 1e-5
            slope = (f(r + h) - f(r - h)) / (2.0 * h)
            out.append((r, eps_xx_rel(r, k_hat, eta, wp2_total, dim).imag / slope))
    return out
