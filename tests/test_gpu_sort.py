"""The re-sort by triangle (fetd_sort) as a permutation: it reorders the
particles in memory and drops the lost ones, and changes nothing a caller
can see.  Checked through the C-ABI on a run whose fast electrons cross
several edges between sorts (some to triangles far away in the Morton
numbering, which the sort handles outside its per-block window) and leave
through the walls: every particle's id, triangle, slot, barycentrics and
momentum read back bit for bit the same across each sort, the lost count
too, with a ragged particle count and in both particle precisions."""
import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I

pytestmark = pytest.mark.gpu


def _fp():
    from paper_1707_04333_amd import fetdpic
    return fetdpic


def _walls(precision, n=100_003, n_side=64, gamma=3.0):
    m = I.grid_mesh(n_side, n_side, 0.1, 0.1, seed=11)
    rng = np.random.default_rng(17)
    tri, lam = I.sample_in_triangles(m, n, rng)
    ang = rng.uniform(0, 2 * np.pi, n)
    um = I.C_LIGHT * np.sqrt(gamma * gamma - 1.0)
    u = np.stack([um * np.cos(ang), um * np.sin(ang)], 1)
    dt = 0.2 * (0.1 / (n_side - 1)) / I.C_LIGHT  # inside the leapfrog limit
    sp = I.Species("electron", -I.E_CHARGE, I.M_E, 1e6, tri, lam, u)
    return I.Workload("walls", m, [sp], dt, 20, "boris", precision, bz_ext=0.2, spai_level=1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sort_is_a_permutation_of_the_live_particles(precision):
    g = _fp().from_workload(_walls(precision), spai_level=1, resort_every=1000)
    lost = []
    for _ in range(6):
        g.step(3, "boris")
        before, d0 = g.particles(0), g.diagnostics()
        g.sort()
        after, d1 = g.particles(0), g.diagnostics()
        for k in ("id", "tri", "slot", "lam", "u"):
            assert np.array_equal(before[k], after[k]), k
        assert d1["n_lost"] == d0["n_lost"]
        lost.append(d1["n_lost"])
    assert lost[0] > 0 and lost[-1] > lost[0]  # particles leave between sorts
    # a sort right after a sort (every particle inside its block's window)
    before = g.particles(0)
    g.sort()
    g.sort()
    after = g.particles(0)
    for k in ("id", "tri", "slot", "lam", "u"):
        assert np.array_equal(before[k], after[k]), k
    assert g.diagnostics()["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6)
    g.close()
