"""The seeded input generators of the tetrahedral workloads: the 3-D
Maxwell-Juttner sampler against the closed-form mean Lorentz factor
<gamma> = 3 theta + K1(1/theta) / K2(1/theta) and against the CDF of
u^2 exp(-gamma/theta) du integrated numerically; positions inside their
tetrahedra; zero net charge and momentum of the pair plasma."""
import numpy as np
import pytest
from scipy import integrate, special

from paper_1707_04333_amd import inputs3 as J


@pytest.mark.parametrize("theta", [0.1, 1.0, 5.0])
def test_mj3d_mean_gamma_closed_form(theta):
    rng = np.random.default_rng(1234)
    u = J.sample_mj3d(400_000, theta, rng)
    g = np.sqrt(1.0 + u * u)
    exact = 3.0 * theta + special.kn(1, 1.0 / theta) / special.kn(2, 1.0 / theta)
    assert abs(g.mean() - exact) <= 5.0 * g.std() / np.sqrt(g.size)


@pytest.mark.parametrize("theta", [0.1, 2.0])
def test_mj3d_cdf(theta):
    """Kolmogorov-Smirnov distance to the numerically integrated CDF."""
    rng = np.random.default_rng(99)
    n = 200_000
    u = np.sort(J.sample_mj3d(n, theta, rng))
    grid = np.linspace(0.0, u[-1] * 1.05, 200_001)
    dens = grid ** 2 * np.exp(-(np.sqrt(1.0 + grid ** 2) - 1.0) / theta)
    cdf = integrate.cumulative_trapezoid(dens, grid, initial=0.0)
    norm = integrate.quad(lambda v: v * v * np.exp(-(np.sqrt(1 + v * v) - 1) / theta), 0, np.inf)[0]
    F = np.interp(u, grid, cdf) / norm
    emp_hi = np.arange(1, n + 1) / n
    emp_lo = np.arange(0, n) / n
    D = max(np.abs(emp_hi - F).max(), np.abs(F - emp_lo).max())
    assert D <= 1.95 / np.sqrt(n), D


def test_pair_plasma_positions_and_neutrality():
    w = J.tet_pair_plasma(n_side=6, length=0.006, n_pairs=5000, theta=0.3)
    e, p = w.species
    assert np.array_equal(e.tri, p.tri) and np.array_equal(e.lam, p.lam)
    assert e.q == -p.q and e.w == p.w
    assert np.abs(e.u + p.u).max() == 0.0
    assert (e.lam >= 0).all() and (e.lam.sum(axis=1) <= 1.0).all()
    assert e.tri.min() >= 0 and e.tri.max() < w.mesh.n_tets
