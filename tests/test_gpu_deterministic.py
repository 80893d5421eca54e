"""The deterministic option (fetd_opts.deterministic): every current
contribution goes into a fixed-point accumulator per edge with integer
atomics, so the step's result does not depend on the order of the adds.
Checked bit for bit through the C-ABI:

* the same run with re-sorts every 3 steps and every 50 steps (different
  particle orders in memory, different tiles);
* batched (graph replay, tile queue) against the same runs stepped one by
  one;
* a run saved after 12 steps (fields_get b, d; particles_get) and resumed
  in a new simulation (fields_load, particles_load_bary) against the run
  that went on;
* the autotuner's trial steps against plain steps;
and against the FP64 oracle within 1e-12 (the accumulator's sum differs
from the oracle's sequential sum by rounding only)."""
import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I

pytestmark = pytest.mark.gpu


def _fp():
    from paper_1707_04333_amd import fetdpic
    return fetdpic


def _wl(n_side=20, length=0.03, n_pairs=9_001, theta=0.3, precision="fp64"):
    return I.pair_plasma(n_side=n_side, length=length, n_pairs=n_pairs, theta=theta, steps=40,
                         precision=precision)


def _state(g, n_species=2):
    out = {name: g.field(name) for name in ("e", "d", "b", "j")}
    for si in range(n_species):
        p = g.particles(si)
        for k in ("id", "tri", "slot", "lam", "u"):
            out[f"{k}{si}"] = p[k]
    return out


def _assert_bitwise(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), (k, float(np.abs(a[k] - b[k]).max()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deterministic_independent_of_sort_order(precision):
    fp = _fp()
    w = _wl(precision=precision)
    a = fp.from_workload(w, spai_level=1, deterministic=True, resort_every=3)
    b = fp.from_workload(w, spai_level=1, deterministic=True, resort_every=50)
    a.step(25, "hc")
    b.step(25, "hc")
    _assert_bitwise(_state(a), _state(b))
    assert a.diagnostics()["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6)
    a.close()
    b.close()


def test_deterministic_matches_oracle(oracle_lib):
    w = _wl()
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = oracle_lib.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1,
                                bz_ext=w.bz_ext)
    g = _fp().from_workload(w, spai_level=1, deterministic=True, resort_every=7)
    osim.step(30, "vay")
    g.step(30, "vay")
    for si, s in enumerate(osim.species):
        gp = g.particles(si)
        alive = np.nonzero(s.tri >= 0)[0]
        assert np.array_equal(gp["id"], alive)
        assert np.array_equal(gp["tri"], s.tri[alive]) and np.array_equal(gp["slot"], s.slot[alive])
        assert np.abs(gp["lam"] - s.lam[alive]).max() <= 1e-12
        assert np.abs(gp["u"] - s.u[alive]).max() <= 1e-12 * np.abs(s.u).max()
    for name, ref in (("e", osim.e), ("d", osim.d), ("b", osim.b), ("j", osim.last_cur)):
        got = g.field(name)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), name
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deterministic_batched_equals_separate(precision):
    fp = _fp()
    specs = [(12, 0.02, 3001, 0.3), (20, 0.03, 9000, 0.1), (9, 0.015, 1500, 1.0)]
    wls = [_wl(n, L, p, t, precision) for n, L, p, t in specs]
    batched = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
               for w in wls]
    single = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
              for w in wls]
    b = fp.Batch(batched, use_graph=True)
    b.step(33, "boris")
    for s in single:
        s.step(33, "boris")
    st = b.stats()
    assert st["graph_captures"] == 1 and st["graph_replays"] >= 2, st
    for gb, gs in zip(batched, single):
        _assert_bitwise(_state(gb), _state(gs))
    b.close()
    for s in batched + single:
        s.close()


def test_batched_members_keep_their_tiles():
    """Runs with different tiles (512, 2048, 1024) in one batch, the tile of
    one member changed between calls (the batch rebuilds its tile list):
    bit for bit the runs stepped one by one, and the batch leaves each
    member's tile as it was set."""
    fp = _fp()
    specs = [(12, 0.02, 3001, 0.3), (20, 0.03, 9000, 0.1), (9, 0.015, 1500, 1.0)]
    tiles = (512, 2048, 1280)
    wls = [_wl(n, L, p, t, "fp64") for n, L, p, t in specs]
    batched = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
               for w in wls]
    single = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
              for w in wls]
    for g, t in zip(batched, tiles):
        g.set_tile(t)
    b = fp.Batch(batched, use_graph=True)
    b.step(20, "vay")
    assert [g.get_tile() for g in batched] == list(tiles)
    batched[2].set_tile(512)
    b.step(13, "vay")
    for s in single:
        s.step(33, "vay")
    assert b.stats()["graph_replays"] >= 1
    for gb, gs in zip(batched, single):
        _assert_bitwise(_state(gb), _state(gs))
    b.close()
    for s in batched + single:
        s.close()


def test_batch_stepped_in_short_calls_captures_a_graph():
    """A batch stepped in calls of two re-sort intervals (2K steps, too few
    for a lead, an eager cycle and a captured cycle in one call) captures
    its graph on a later call and replays it; a call of K steps between
    replays (one sort: the buffers' parity flips) and a change of pusher
    each make it capture again; the runs stay bit for bit the runs stepped
    one by one."""
    fp = _fp()
    specs = [(12, 0.02, 3001, 0.3), (16, 0.025, 6000, 0.1)]
    wls = [_wl(n, L, p, t, "fp64") for n, L, p, t in specs]
    K = 6
    batched = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=K)
               for w in wls]
    single = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=K)
              for w in wls]
    b = fp.Batch(batched, use_graph=True)
    plan = [("hc", 3), ("hc", 2 * K), ("hc", 2 * K), ("hc", 2 * K), ("hc", K), ("hc", 2 * K),
            ("vay", 2 * K), ("vay", 2 * K), ("vay", 2 * K + 5)]
    for pusher, n in plan:
        b.step(n, pusher)
        for s in single:
            s.step(n, pusher)
    st = b.stats()
    assert st["graph_captures"] >= 3 and st["graph_replays"] >= 4, st
    for gb, gs in zip(batched, single):
        _assert_bitwise(_state(gb), _state(gs))
    b.close()
    for s in batched + single:
        s.close()


def test_deterministic_save_and_resume():
    fp = _fp()
    w = _wl()
    ref = fp.from_workload(w, spai_level=1, deterministic=True, resort_every=5)
    ref.step(12, "hc")
    b, d = ref.field("b"), ref.field("d")
    parts = [ref.particles(si) for si in range(2)]
    ref.step(13, "hc")
    sim = fp.Sim(w.mesh, w.dt, I.EPS0, I.MU0, I.C_LIGHT, precision="fp64", spai_level=1,
                 deterministic=True, resort_every=5)
    sim.fields_set(bz_ext=np.full(w.mesh.n_tris, float(w.bz_ext)))
    sim.fields_load(b=b, d=d)
    for s, p in zip(w.species, parts):
        sim.load(s.q, s.m, s.w, p["tri"], p["lam"], p["u"], slot=p["slot"])
    sim.step(13, "hc")
    a, r = _state(sim), _state(ref)
    # the resumed run numbers its particles by their rank among the saved ones
    for si in range(2):
        a[f"id{si}"] = parts[si]["id"][a[f"id{si}"]]
    _assert_bitwise(a, r)
    ref.close()
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_returns_argmin_and_keeps_the_run(precision):
    """fetd_autotune picks the tile, the scan width, the exit mode (FP32
    particles) and then the re-sort interval of least measured cost, and its
    trial steps are ordinary steps of the run: in deterministic mode the
    state equals, bit for bit, that of a plain run of as many steps (7 x 20
    tile trials, 3 x 20 scan trials, FP32: 2 x 20 exit-mode trials, 40
    cadence trials)."""
    fp = _fp()
    w = _wl(n_side=24, length=0.038, n_pairs=40_000, precision=precision)
    tuned = fp.from_workload(w, precision=precision, spai_level=1, deterministic=True)
    plain = fp.from_workload(w, precision=precision, spai_level=1, deterministic=True)
    r = tuned.autotune("boris", trial_steps=40, with_costs=True)
    cands = [c for c in (5, 10, 20, 40, 80, 160) if c <= 40]
    assert set(r["costs"]) == set(cands)
    assert all(v > 0 for v in r["costs"].values())
    assert r["resort_every"] == min(cands, key=lambda c: r["costs"][c])
    tc = r["tile_costs"]
    assert set(tc) == set(range(512, 2049, 256)) and all(v > 0 for v in tc.values())
    assert r["tile"] == min(tc, key=lambda c: tc[c]) and tuned.get_tile() == r["tile"]
    sc = r["scan_costs"]
    assert set(sc) == {64, 16, 8} and all(v > 0 for v in sc.values())
    assert r["scan"] == min(sc, key=lambda c: sc[c]) and tuned.get_scan() == r["scan"]
    dc = r["defer_costs"]
    if precision == "fp64":
        assert dc == {} and r["defer_exits"] == 1 and tuned.get_defer_exits() == 1
    else:
        assert set(dc) == {0, 1} and all(v > 0 for v in dc.values())
        assert r["defer_exits"] == min(dc, key=lambda c: dc[c])
        assert tuned.get_defer_exits() == r["defer_exits"]
    plain.step((10 if precision == "fp64" else 12) * 20 + 40, "boris")
    _assert_bitwise(_state(tuned), _state(plain))
    tuned.step(7, "boris")
    plain.step(7, "boris")
    _assert_bitwise(_state(tuned), _state(plain))
    tuned.close()
    plain.close()


@pytest.mark.parametrize("precision", ["mixed", "mixed_f64field"])
def test_deferred_exits_give_the_same_run(precision):
    """Deterministic mode, FP32 particles: deferred exits (stays decided by
    comparison with a margin, the others traced from the start after the
    pass) give bit for bit the run with every first piece traced in the
    pass: the same stays, the same arithmetic (hot plasma, re-sorts,
    crossings, 40 steps); FP64 always defers and ignores the switch."""
    fp = _fp()
    w = _wl(n_side=24, length=0.038, n_pairs=40_000, precision="mixed")
    a = fp.from_workload(w, precision=precision, spai_level=1, deterministic=True, resort_every=7)
    b = fp.from_workload(w, precision=precision, spai_level=1, deterministic=True, resort_every=7)
    assert a.get_defer_exits() == 0
    b.set_defer_exits(1)
    assert b.get_defer_exits() == 1
    a.step(40, "hc")
    b.step(40, "hc")
    _assert_bitwise(_state(a), _state(b))
    assert a.diagnostics()["n_segments"] == b.diagnostics()["n_segments"]
    with pytest.raises(Exception):
        b.set_defer_exits(2)
    a.close()
    b.close()


@pytest.mark.parametrize("tile,scan", [(512, 64), (2048, 8), (1024, 16), (1280, 8), (1792, 16)])
def test_every_tile_gives_the_same_run(tile, scan):
    """Deterministic mode: a run at each tile size and scan width equals the
    run at the defaults bit for bit (hot plasma, re-sorts, crossings)."""
    fp = _fp()
    w = _wl(n_side=24, length=0.038, n_pairs=40_000)
    a = fp.from_workload(w, spai_level=1, deterministic=True, resort_every=7)
    b = fp.from_workload(w, spai_level=1, deterministic=True, resort_every=7)
    assert a.get_tile() == 1024 and a.get_scan() == 64
    b.set_tile(tile)
    b.set_scan(scan)
    assert b.get_tile() == tile and b.get_scan() == scan
    a.step(30, "hc")
    b.step(30, "hc")
    _assert_bitwise(_state(a), _state(b))
    for bad in (640, 256, 2304):
        with pytest.raises(Exception):
            b.set_tile(bad)
    with pytest.raises(Exception):
        b.set_scan(32)
    a.close()
    b.close()
