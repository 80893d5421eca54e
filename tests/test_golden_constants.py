"""Pin the physical constants both sides use (CODATA-2018, passed in by
the seeded workload module) to the worked values the paper prints, and
the mesh-count convention to the paper's Bernstein mesh."""
import json
import math
import os

import pytest

from paper_1707_04333_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _agree(x, ref, digits):
    """Within one unit of the last printed digit (the paper truncates)."""
    mant = abs(ref) / 10 ** math.floor(math.log10(abs(ref)))
    return abs(x - ref) <= abs(ref) * 10 ** (1 - digits) / mant


def test_synchrocyclotron_field():
    g = GOLD["synchrocyclotron_Bz"]
    bz = I.M_E * g["v0"] / (I.E_CHARGE * g["r"])
    assert _agree(bz, g["value"], g["digits"])
    f = I.E_CHARGE * bz / (2 * math.pi * I.M_E)
    assert _agree(f, GOLD["synchrocyclotron_rf"]["value"], GOLD["synchrocyclotron_rf"]["digits"])


def test_bernstein_parameters():
    g = GOLD["bernstein_nonrel_omega_c"]
    assert _agree(I.E_CHARGE * g["B0"] / I.M_E, g["value"], g["digits"])
    g = GOLD["bernstein_pair_omega_c"]
    wc = I.E_CHARGE * g["B0"] / I.M_E
    assert _agree(wc, g["value"], g["digits"])
    wp = 3.0 * wc
    assert _agree(wp, GOLD["bernstein_pair_omega_p"]["value"], 5)
    n = wp * wp * I.EPS0 * I.M_E / I.E_CHARGE ** 2
    assert _agree(n, GOLD["bernstein_pair_density"]["value"], 5)


def test_mesh_euler_convention():
    """The paper's counts are of a disk (chi = 1); our edge/face counting
    convention gives the same characteristic for a square mesh."""
    g = GOLD["bernstein_mesh_euler"]
    assert g["nodes"] - g["edges"] + g["faces"] == g["chi"]
    import oracle
    m = I.grid_mesh(11, 9, 1.0, 1.0)
    T = oracle.Topology(m.node_xy, m.tri_nodes)
    assert T.nn - T.ne + T.nf == g["chi"]


def test_light_speed_consistency():
    """c, eps0 and mu0 are CODATA-2018 values; 1/sqrt(eps0 mu0) = c to 1e-9."""
    assert abs(1 / math.sqrt(I.EPS0 * I.MU0) / I.C_LIGHT - 1) < 1e-9
