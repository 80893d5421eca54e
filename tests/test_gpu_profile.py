"""Stage timing through the C-ABI (fetd_profile_mask, fetd3_profile_mask):
a mask times only its stages, a sampling period only the steps whose index
is its multiple, the events carried by the kernel dispatches give one
positive interval per launch, and the timed stages, which run one after
another on one stream, never add up to more than the run's wall time."""
import time

import pytest

from paper_1707_04333_amd import inputs as I
from paper_1707_04333_amd import inputs3 as J

pytestmark = pytest.mark.gpu


def _timed(sim, n):
    t0 = time.perf_counter()
    sim.step(n, "boris")
    sim.sync()
    return (time.perf_counter() - t0) * 1e3


def test_stage_mask_triangles():
    from paper_1707_04333_amd import fetdpic as fp
    w = I.pair_plasma(n_side=24, length=0.038, n_pairs=20_000, theta=0.3, steps=40)
    sim = fp.from_workload(w, precision="mixed", spai_level=1)
    sim.set_resort(5)
    sim.step(3, "boris")
    sim.sync()
    sim.profile(stages=["particles"])
    _timed(sim, 10)
    st = sim.stage_times()
    assert st["particles"][1] == 10 * len(w.species) and st["particles"][0] > 0
    for k in ("faraday", "ampere", "spmv", "sort"):
        assert st[k] == (0.0, 0), k
    sim.profile(True)
    wall = _timed(sim, 10)
    st = sim.stage_times()
    for k in ("faraday", "ampere", "spmv"):
        assert st[k][1] == 10 and st[k][0] > 0, k
    assert st["particles"][1] == 10 * len(w.species)
    assert st["sort"][1] >= 1 and st["sort"][0] > 0
    assert sum(v[0] for v in st.values()) <= wall
    s0 = sim.diagnostics()["step"]
    sim.profile(stages=["particles"], every=4)
    _timed(sim, 12)
    st = sim.stage_times()
    sampled = sum(1 for k in range(s0, s0 + 12) if k % 4 == 0)
    assert st["particles"][1] == sampled * len(w.species) and st["particles"][0] > 0
    assert st["faraday"] == (0.0, 0)
    sim.profile(False)
    _timed(sim, 5)
    assert all(v == (0.0, 0) for v in sim.stage_times().values())
    assert sim.diagnostics()["gauss_rel"] <= 1e-12
    sim.close()


def test_stage_mask_tetrahedra():
    from paper_1707_04333_amd import fetd3
    w = J.tet_pair_plasma(n_side=6, length=0.006, n_pairs=3001, theta=0.3)
    sim = fetd3.from_workload3(w, resort_every=5, precision="mixed")
    sim.step(3, "boris")
    sim.sync()
    sim.profile(stages=["particles", "sort"])
    _timed(sim, 10)
    st, n = sim.stage_times()
    assert n == 10 * len(w.species) and st["particles"] > 0 and st["sort"] > 0
    assert st["faraday"] == st["ampere"] == st["spmv"] == 0.0
    sim.profile(True)
    wall = _timed(sim, 10)
    st, n = sim.stage_times()
    assert n == 10 * len(w.species)
    assert min(st.values()) > 0 and sum(st.values()) <= wall
    s0 = sim.diagnostics()["step"]
    sim.profile(stages=["particles"], every=3)
    _timed(sim, 10)
    st, n = sim.stage_times()
    assert n == sum(1 for k in range(s0, s0 + 10) if k % 3 == 0) * len(w.species)
    assert st["particles"] > 0 and st["faraday"] == st["sort"] == 0.0
    sim.profile(False)
    d = sim.diagnostics()
    assert d["gauss_rel"] <= 1e-12 and d["divb_rel"] <= 1e-13
    sim.close()
