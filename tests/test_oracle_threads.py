"""The oracle's timing mode (particle stage over OpenMP threads, private
currents added in thread order) computes the same step as its parity mode:
every particle's update is the same arithmetic, only the order of the
current sums differs."""
import numpy as np

from paper_1707_04333_amd import inputs as I


def test_threaded_oracle_matches_single_thread(oracle_lib):
    w = I.pair_plasma(n_side=16, length=0.025, n_pairs=20_003, theta=0.5, steps=10,
                      precision="fp64")
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    one = oracle_lib.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1,
                               bz_ext=w.bz_ext)
    many = oracle_lib.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1,
                                bz_ext=w.bz_ext)
    one.step(6, "vay")
    many.step(6, "vay", threads=5)
    for a, b in zip(one.species, many.species):
        assert np.array_equal(a.tri, b.tri) and np.array_equal(a.slot, b.slot)
        assert np.abs(a.lam - b.lam).max() <= 1e-12
        assert np.abs(a.u - b.u).max() <= 1e-12 * np.abs(a.u).max()
    assert np.abs(one.e - many.e).max() <= 1e-12 * np.abs(one.e).max()
    assert one.segments == many.segments
