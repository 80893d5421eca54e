"""Benchmark: particle-steps/s of the full PIC step on one MI355X.

Default workload (the ``value`` line): the large single run — a graded
jittered Delaunay mesh of the unit square (708 x 708 nodes, element size
ratio 10, 1,000,000 triangles) with PEC walls and a matched absorbing outer
layer, 128M electrons (95% in-plane Maxwell-Juttner at kT/mc^2 = 0.5, 5% a
gamma = 20 beam), uniform B0 = 1 T with omega_c/omega_p = 2, Higuera-Cary
pusher, particles re-sorted by triangle every 20 steps.  ``value`` is the
FP64 path (every stage in FP64, the paper's precision); the two mixed forms
(FP32 particle state with FP32 or FP64 fields; FP64 current accumulation
and Gauss accounting) are reported beside it on the same workload.

A step is one pass of the whole path: Faraday + field record, the fused
gather/push/track/deposit stage, Ampere, the SPAI SpMV, and the counting
sort when due.  The timed window starts at a step that sorts, so it holds
ceil(steps/K) sorts (K = the re-sort interval): the sort's cost is inside
``value``.  Inputs are resident in HBM before the timed region.

Beside it: the pair-plasma Bernstein run (199,712 triangles, 16M
particles) in FP64 and mixed, the batched sweep (64 independent uneven
runs, one launch per phase per step, graph replay over whole re-sort
cycles) against the same runs stepped one by one, the fused particle kernel
on the HBM roofline from HIP events that its launches on every 7th step of
the timed region carry in their own dispatches, a plain device-to-device
copy as the measured bandwidth ceiling, and the FP64 CPU oracle on a
bounded sample of the headline workload on all host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload large|pair|boosted|cyclotron|bernstein|synchro|tet]
                       [--timing-overhead]
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec + achieved HBM GB/s; mixed/batched vs FP64 at Gauss residual"
HBM_PEAK_GBS = 8000.0
DEFAULT_PAIRS = 8_000_000
KERNEL_SRC = os.path.join(ROOT, "paper_1707_04333_amd", "csrc", "fetd_particles.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_particle_step_large_graded_traffic.json")
ISSUE_FILE = os.path.join(ROOT, "profiles", "k_particle_step_large_graded_issue.json")
# VALU issue ceiling: 256 CUs x 4 SIMDs, one wavefront-instruction (64 lanes
# on a 16-lane SIMD: 4 cycles) per SIMD every 4 cycles at the 2.4 GHz peak
# engine clock.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
PAIR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_particle_step_pair_plasma_traffic.json")
KERNEL3_SRC = os.path.join(ROOT, "paper_1707_04333_amd", "csrc", "fetd3_kernels.hip")
TRAFFIC3_FILE = os.path.join(ROOT, "profiles", "k3_particles_tet_pair_plasma_traffic.json")
# Inside the timed region the particle launches of every TIMING_EVERY-th step
# carry HIP events; 7 is coprime with every re-sort interval used (5 * 2^k),
# so the sampled steps fall on every phase of the sort cycle.
TIMING_EVERY = 7
LARGE_RESORT = 20


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def particle_launch_bytes(n_particles, nf, ne, fp32):
    """Algorithmic bytes of one fused particle-stage launch: every particle
    reads and writes its state (key 4 B, barycentric pair and momentum
    2 x 2 reals), every triangle's field record (32 B), gradients (6 reals,
    padded to 8 in FP32), edge and neighbour tables (16 B each) are read
    once, and every edge's FP64 current is read and written once."""
    r = 4 if fp32 else 8
    per_particle = 2 * (4 + 4 * r)
    per_tri = 32 + (8 if fp32 else 6) * r + 16 + 16
    return n_particles * per_particle + nf * per_tri + ne * 16


def kernel_hash(src=KERNEL_SRC):
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _same_launch(leg, tile, scan, defer=None):
    """A counter record applies to a leg run at the same tile, scan width
    and exit mode (when the record states them)."""
    return ((tile is None or leg.get("tile") in (None, tile)) and
            (scan is None or leg.get("scan") in (None, scan)) and
            (defer is None or leg.get("defer_exits") in (None, defer)))


def measured_traffic(precision, traffic_file=TRAFFIC_FILE, src=KERNEL_SRC, tile=None, scan=None,
                     defer=None):
    """HBM bytes per particle launch from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or None when
    the kernel source changed since they were taken or they were taken at
    another tile or scan width."""
    try:
        rec = json.load(open(traffic_file))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_hash(src):
        return None
    leg = rec.get(precision, {})
    return leg.get("hbm_bytes_per_launch") if _same_launch(leg, tile, scan, defer) else None


def measured_valu(precision, issue_file=ISSUE_FILE, src=KERNEL_SRC, tile=None, scan=None,
                  defer=None):
    """VALU instructions (wavefront instructions) per particle launch from
    the committed SQ counter runs, or None when the kernel source changed
    since they were taken or they were taken at another tile or scan."""
    try:
        rec = json.load(open(issue_file))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_hash(src):
        return None
    leg = rec.get(precision, {})
    return leg.get("valu_per_launch") if _same_launch(leg, tile, scan, defer) else None


def host_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_threads():
    """Threads of the oracle's timing mode: OMP_NUM_THREADS if set, else the
    CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return host_info()["affinity_cpus"] or 1


def copy_ceiling_gbs(nbytes=1 << 30, reps=5):
    """Measured device-to-device copy bandwidth (read + write bytes per
    second) of the library's plain copy kernel over 1 GiB buffers: the
    achievable HBM ceiling."""
    from paper_1707_04333_amd import fetdpic as fp
    return fp.copy_ceiling(0, nbytes, reps)


def run_gpu(w, precision, steps, warmup, pusher, resort=None, pin=(None, None, None)):
    """One workload in one precision.  The autotuner chooses the particle
    tile and scan width (unless `pin` fixes them), and the re-sort interval
    unless `resort` fixes it.  The timed window starts at a sorting step
    and covers `steps` steps (inputs already on the device)."""
    from paper_1707_04333_amd import fetdpic as fp
    log(f"{precision}: creating simulation ({w.n_particles} particles)")
    t0 = time.perf_counter()
    sim = fp.from_workload(w, precision=precision, spai_level=w.spai_level, device=0,
                           resort_every=resort or 20)
    log(f"{precision}: created in {time.perf_counter() - t0:.1f} s")
    info = sim.info()
    sim.diagnostics()  # Gauss baseline at step 0
    tuned = sim.autotune(pusher, trial_steps=160 if resort is None else 20, with_costs=True)
    if resort is None:
        resort = tuned["resort_every"]
    else:
        sim.set_resort(resort)
    if pin[0]:
        sim.set_tile(pin[0])
        tuned["tile"] = pin[0]
    if pin[1]:
        sim.set_scan(pin[1])
        tuned["scan"] = pin[1]
    if pin[2] is not None and precision != "fp64":
        sim.set_defer_exits(pin[2])
        tuned["defer_exits"] = pin[2]
    log(f"{precision}: tile {tuned['tile']}, scan {tuned['scan']} lanes, exits "
        f"{'deferred' if tuned['defer_exits'] or precision == 'fp64' else 'traced'}, "
        f"re-sort every {resort}" + (" (pinned)" if pin[0] or pin[1] or pin[2] is not None
                                     else ""))
    # the autotuner leaves the order decayed: the next step sorts
    align = 0
    # warm-up: at least `warmup` steps, ending where the next step sorts
    w_steps = align + int(math.ceil(max(warmup, 1) / resort)) * resort
    sim.step(w_steps, pusher)
    sim.sync()
    # the timed region times the particle kernel only, on every
    # TIMING_EVERY-th step (a dispatch that carries events idles the device
    # for several microseconds around it)
    sim.profile(stages=["particles"], every=TIMING_EVERY)
    t0 = time.perf_counter()
    sim.step(steps, pusher)
    sim.sync()
    t1 = time.perf_counter()
    particles = sim.stage_times()["particles"]
    log(f"{precision}: {steps} steps in {t1 - t0:.3f} s")
    # stage breakdown: every stage timed over whole re-sort intervals
    stage_steps = resort * max(1, int(math.ceil(100 / resort)))
    back = (resort - steps % resort) % resort  # back to a sort boundary
    if back:
        sim.step(back, pusher)
    sim.profile(True)
    sim.step(stage_steps, pusher)
    stages = sim.stage_times()
    sim.profile(False)
    diag = sim.diagnostics()
    sim.close()
    return dict(elapsed=t1 - t0, particles=particles, stages=stages, stage_steps=stage_steps,
                diag=diag, info=info, resort=resort, warmup_steps=w_steps,
                sorts_timed=int(math.ceil(steps / resort)), tile=tuned["tile"],
                scan=tuned["scan"], defer=int(tuned["defer_exits"] or precision == "fp64"))


def leg_record(r, n_p, steps, species_n, fp32, traffic=None, valu=None):
    """JSON record of one precision leg: throughput, the particle kernel's
    algorithmic bandwidth, the per-stage breakdown and the Gauss residual."""
    nf, ne = r["info"]["n_tris"], r["info"]["n_edges"]
    ms, launches = r["particles"]
    per_launch = float(np.mean([particle_launch_bytes(n, nf, ne, fp32) for n in species_n]))
    avg_s = ms / 1e3 / max(launches, 1)
    achieved = per_launch / avg_s / 1e9
    return {"value": n_p * steps / r["elapsed"], "ms_per_step": r["elapsed"] / steps * 1e3,
            "gauss_rel": r["diag"]["gauss_rel"], "resort_every": r["resort"],
            "tile": r["tile"], "scan_lanes": r["scan"], "defer_exits": r["defer"],
            "sorts_in_timed_steps": r["sorts_timed"],
            "roofline": {"bound": "hbm", "kernel": "k_particle_step", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic, "avg_launch_ms": avg_s * 1e3,
                         "algorithmic_bytes_per_launch": per_launch},
            "valu_issue": None if valu is None else {
                "instr_per_launch": valu, "peak_per_s": VALU_ISSUE_PEAK,
                "frac": valu / avg_s / VALU_ISSUE_PEAK},
            "stage_ms_per_step": {k: v[0] / r["stage_steps"] for k, v in r["stages"].items()},
            "hbm_gbs_step": sum(particle_launch_bytes(n, nf, ne, fp32) for n in species_n)
            / (r["elapsed"] / steps) / 1e9}


def run_timing_overhead(args, window=160, reps=2):
    """What stage timing costs the step: the 16M-particle pair plasma
    (mixed, Boris, re-sort every 160 steps, so every window holds one sort)
    stepped in windows of 160 steps with nothing timed, with the particle
    stage timed on every TIMING_EVERY-th step (the timed region's setting),
    on every step, and with every stage timed on every step; 50 ms of idle
    between windows lets a kernel trace tell them apart."""
    from paper_1707_04333_amd import fetdpic as fp
    from paper_1707_04333_amd import inputs as I
    log("timing overhead: generating the pair plasma")
    w = I.pair_plasma(n_pairs=args.pairs, theta=args.theta, precision="mixed")
    sim = fp.from_workload(w, precision="mixed", spai_level=1, device=0)
    sim.set_resort(window)
    sim.step(args.warmup, "boris")
    sim.sync()
    modes = (("untimed", None), ("particles_every_%d" % TIMING_EVERY, (["particles"], TIMING_EVERY)),
             ("particles_every_step", (["particles"], 1)), ("all_stages_every_step", (None, 1)))
    out = {k: [] for k, _ in modes}
    for _ in range(reps):
        for name, mode in modes:
            time.sleep(0.05)
            if mode is not None:
                sim.profile(stages=mode[0], every=mode[1])
            t0 = time.perf_counter()
            sim.step(window, "boris")
            sim.sync()
            out[name].append((time.perf_counter() - t0) / window * 1e3)
            sim.profile(False)
            log(f"timing overhead: {name} {out[name][-1]:.4f} ms per step")
    sim.close()
    base = min(out["untimed"])
    return {"metric": "ms per step by stage-timing mode", "unit": "ms",
            "workload": "pair plasma, 199,712 triangles, 16M particles, mixed, Boris",
            "window_steps": window, "ms_per_step": {k: min(v) for k, v in out.items()},
            "all_windows": out,
            "overhead_vs_untimed": {k: min(v) / base - 1.0 for k, v in out.items()}}


def run_batched(pusher, min_steps=100, precision="mixed"):
    """64 uneven pair-plasma runs: batched with graph replay, timed over
    whole replayed cycles of two re-sort intervals, against the same runs
    stepped one by one for the same number of steps."""
    from paper_1707_04333_amd import fetdpic as fp
    from paper_1707_04333_amd import inputs as I
    log(f"batched ({precision}): generating 64 runs")
    wls = I.batched_sweep(precision="fp64" if precision == "fp64" else "mixed")
    n_p = sum(w.n_particles for w in wls)
    n_f = sum(w.mesh.n_tris for w in wls)
    species_n = [[sp.n for sp in w.species] for w in wls]
    sims = [fp.from_workload(w, precision=precision, spai_level=1, device=0) for w in wls]
    del wls
    # the persistent particle launch of a step covers every (run, species)
    # segment: its algorithmic bytes are the sum of the segments' launches
    launch_bytes = 0
    for s, ns in zip(sims, species_n):
        inf = s.info()
        launch_bytes += sum(particle_launch_bytes(n, inf["n_tris"], inf["n_edges"],
                                                  precision != "fp64")
                            for n in ns)
    ks = []
    for s in sims:
        s.diagnostics()
        ks.append(s.autotune(pusher, trial_steps=80))
    K = int(np.median(ks))
    for s in sims:
        s.set_resort(K)
    log(f"batched: {n_p} particles on {n_f} triangles, re-sort every {K}")
    b = fp.Batch(sims, use_graph=True)
    # after the autotuner every run sorts next: an eager cycle, then the
    # capture and a first replay
    b.step(4 * K, pusher)
    sims[0].sync()
    st0 = b.stats()
    cycles = max(1, int(math.ceil(min_steps / (2 * K))))
    steps = 2 * K * cycles
    t0 = time.perf_counter()
    b.step(steps, pusher)
    sims[0].sync()
    t_b = time.perf_counter() - t0
    st1 = b.stats()
    replays = st1["graph_replays"] - st0["graph_replays"]
    eager = st1["eager_steps"] - st0["eager_steps"]
    b.close()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s in sims:
            s.step(1, pusher)
    sims[0].sync()
    t_s = time.perf_counter() - t0
    gauss = max(s.diagnostics()["gauss_rel"] for s in sims)
    for s in sims:
        s.close()
    log(f"batched: {steps} steps in {t_b:.3f} s ({replays} graph replays, {eager} eager steps), "
        f"separate {t_s:.3f} s")
    return {"workload": "batched_sweep_64", "n_runs": 64, "n_particles": n_p,
            "n_tris": n_f, "precision": precision, "value": n_p * steps / t_b,
            "ms_per_step": t_b / steps * 1e3, "steps": steps, "graph_replays": replays,
            "eager_steps_timed": eager, "separate_value": n_p * steps / t_s,
            "batched_vs_separate": t_s / t_b, "resort_every": K, "gauss_rel": gauss,
            "particle_launch_algorithmic_bytes": launch_bytes,
            "particle_bytes_gbs_step": launch_bytes / (t_b / steps) / 1e9}


def cpu_baseline(w, pusher, steps=2, absorber=True):
    """The FP64 oracle (its OpenMP timing mode: particles in contiguous
    chunks over all host threads, private currents added in thread order;
    the field update single-threaded) on the same workload: every particle,
    `steps` steps after one warm-up step."""
    import oracle
    from paper_1707_04333_amd import inputs as I
    threads = oracle_threads()
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    t0 = time.perf_counter()
    osim = oracle.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT,
                            spai_level=w.spai_level, bz_ext=w.bz_ext or None)
    if absorber and "sigma_tri" in w.extra:
        damp, damp_b, _ = oracle.absorber_damp(osim.T, w.extra["sigma_tri"], w.dt, I.EPS0)
        osim.damp, osim.damp_b = np.ascontiguousarray(damp), np.ascontiguousarray(damp_b)
    setup = time.perf_counter() - t0
    osim.step(1, pusher, threads=threads)
    t0 = time.perf_counter()
    osim.step(steps, pusher, threads=threads)
    el = time.perf_counter() - t0
    n = sum(s.n for s in osim.species)
    info = host_info()
    return {"value": n * steps / el, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle", "host": info,
            "sample": (f"the same workload ({w.mesh.n_tris} triangles, all {n} particles), "
                       f"{steps} FP64 steps after 1 warm-up step, oracle particle stage on "
                       f"{threads} OpenMP threads ({info['cpu_model']}), field update "
                       f"single-threaded; {el:.1f} s timed, {setup:.1f} s setup")}


def run_synchro(args):
    """The synchrocyclotron of Sec. III.A (one electron, RF gap driven from
    the host every step): steps/s of the driven run, energy gained and the
    Gauss residual.  --workload synchro[_synched|_unsynched|_nonrel]."""
    from paper_1707_04333_amd import experiments as X
    from paper_1707_04333_amd import inputs as I
    case = args.workload.split("_", 1)[1] if "_" in args.workload else "synched"
    w = I.synchrocyclotron(case)
    steps = args.steps if args.steps != 200 else 5000
    t0 = time.perf_counter()
    r = X.run_synchrocyclotron(w, steps, record_every=max(steps // 10, 1))
    el = time.perf_counter() - t0
    return {"metric": METRIC, "value": steps / el, "unit": "particle-steps/s", "n_gpus": 1,
            "steps": steps, "warmup": 0, "ms_per_step": el / steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "synchrocyclotron", "case": case, "n_tris": w.mesh.n_tris,
                       "n_particles": 1, "pusher": "boris_tan", "precision": "fp64"},
            "ekin_eV": [float(e / I.E_CHARGE) for e in r["ekin"]],
            "gauss_rel": r["diag"]["gauss_rel"],
            "note": "one electron; each step reads the electron back to drive the RF phase"}


def run_bernstein(args):
    """The dispersion run of Sec. III.C at v_th = 0.07c: pair plasma on a
    thin periodic strip (6848 triangles, 2.7M particles, mixed precision),
    E_x probed on a line every 16 steps for 32,768 steps; particle-steps/s
    of the probed run and the deviation of the first-band ridge from the
    non-relativistic Bernstein relation."""
    from paper_1707_04333_amd import dispersion as D
    from paper_1707_04333_amd import fetdpic as fp
    from paper_1707_04333_amd import inputs as I
    w = I.bernstein_strip()
    sim = fp.from_workload(w, precision="mixed")
    nx, every = 428, 16
    steps = args.steps if args.steps != 200 else 32768
    lx, ly = w.extra["length_x"], w.extra["length_y"]
    xy = np.stack([(np.arange(nx) + 0.5) * lx / nx, np.full(nx, 0.5 * ly)], axis=1)
    sim.probe_set(xy, every=every, max_samples=steps // every)
    sim.set_resort(20)
    sim.step(64, "boris")
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps - 64, "boris")
    sim.sync()
    el = time.perf_counter() - t0
    samples = sim.probe_get()
    gauss = sim.diagnostics()["gauss_rel"]
    sim.close()
    wc = w.extra["omega_c"]
    k, om, p = D.spectrum(samples, every * w.dt, lx / nx, wc, I.C_LIGHT)
    sel = (k > 0.9) & (k < 38.0)
    theory = D.bernstein_modes(k[sel], np.sqrt(w.extra["theta"]),
                               2.0 * (w.extra["omega_p"] / wc) ** 2, bands=(1,))[0]
    dev = np.abs(D.ridge(k, om, p, 1)[sel] - theory)
    n_p = w.n_particles
    return {"metric": METRIC, "value": n_p * (steps - 64) / el, "unit": "particle-steps/s",
            "n_gpus": 1, "steps": steps - 64, "warmup": 64,
            "ms_per_step": el / (steps - 64) * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 particle state/push/track, f64 deposit+fields", "data": "synthetic",
            "config": {"workload": "bernstein_strip", "n_tris": w.mesh.n_tris,
                       "n_particles": n_p, "theta": w.extra["theta"], "pusher": "boris",
                       "precision": "mixed", "probes": nx, "probe_every": every},
            "gauss_rel": gauss, "band1_median_dw": float(np.median(dev)),
            "band1_frac_within_0.05": float(np.mean(dev < 0.05))}


def tet_particle_launch_bytes(n_particles, nt, ne, fp32):
    """Algorithmic bytes of one tetrahedral particle launch: every particle
    reads and writes its key (4 B), stored barycentric triple and momentum
    (3 + 3 reals); every tetrahedron's gather record (24 reals), gradients
    (12 reals), edge table (32 B), neighbour table (16 B) and node map (4 B)
    are read once; every edge's FP64 current is read and written once."""
    r = 4 if fp32 else 8
    return n_particles * 2 * (4 + 6 * r) + nt * (36 * r + 32 + 16 + 4) + ne * 16


def _run_tet_one(w, precision, steps, warmup, resort_every):
    from paper_1707_04333_amd import fetd3
    t0 = time.perf_counter()
    sim = fetd3.from_workload3(w, resort_every=resort_every, precision=precision)
    log(f"{precision}: simulation created in {time.perf_counter() - t0:.1f} s")
    sim.step(warmup, "boris")
    sim.sync()
    log(f"{precision}: {warmup} warm-up steps done")
    sim.profile(stages=["particles"], every=TIMING_EVERY)
    t0 = time.perf_counter()
    sim.step(steps, "boris")
    sim.sync()
    el = time.perf_counter() - t0
    log(f"{precision}: {steps} steps in {el:.3f} s")
    particle_ms, launches = sim.stage_times()
    particle_ms = particle_ms["particles"]
    # stage breakdown from a separate pass (every stage timed)
    stage_steps = min(steps, 100)
    sim.profile(True)
    sim.step(stage_steps, "boris")
    stages, _ = sim.stage_times()
    sim.profile(False)
    d = sim.diagnostics()
    sim.close()
    return el, particle_ms, launches, {k: v / stage_steps for k, v in stages.items()}, d


def run_tet(args):
    """The tetrahedral path on a triply periodic pair plasma: 48^3 Kuhn cells
    (663,552 tetrahedra), 8M electrons + 8M positrons (24 per tetrahedron),
    3-D Maxwell-Juttner momenta at theta = 0.1, B0 = 1 T along z,
    omega_c/omega_p = 2, Boris, sorted every 10 steps (the best of 10, 20,
    40, 80 measured on this workload); mixed precision (the value) and FP64."""
    from paper_1707_04333_amd import inputs3 as J
    log("generating the tetrahedral pair plasma")
    w = J.tet_pair_plasma(n_pairs=args.pairs)
    log(f"generated {w.mesh.n_tets} tetrahedra and {w.n_particles} particles")
    n_p = w.n_particles
    resort = 10
    species_n = [s.n for s in w.species]
    nt = w.mesh.n_tets
    res = {}
    for prec in ("mixed", "fp64"):
        if prec == "fp64" and args.no_fp64:
            continue
        log(f"tetrahedral run, {prec}")
        el, particle_ms, launches, stages, d = _run_tet_one(w, prec, args.steps, args.warmup,
                                                            resort)
        ne = d["n_edges"]
        per_launch = float(np.mean([tet_particle_launch_bytes(n, nt, ne, prec == "mixed")
                                    for n in species_n]))
        avg_s = particle_ms / 1e3 / max(launches, 1)
        achieved = per_launch / avg_s / 1e9
        res[prec] = {"value": n_p * args.steps / el, "ms_per_step": el / args.steps * 1e3,
                     "roofline": {"bound": "hbm", "kernel": "k3_particles", "achieved": achieved,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": achieved / HBM_PEAK_GBS,
                                  "traffic": (measured_traffic(prec, TRAFFIC3_FILE, KERNEL3_SRC)
                                              if args.pairs == DEFAULT_PAIRS else None),
                                  "avg_launch_ms": avg_s * 1e3,
                                  "algorithmic_bytes_per_launch": per_launch},
                     "stage_ms_per_step": stages,
                     "gauss_rel": d["gauss_rel"], "divb_rel": d["divb_rel"],
                     "pieces_per_particle_step": d["n_segments"]
                     / (n_p * (args.steps + args.warmup + min(args.steps, 100))),
                     "n_edges": ne,
                     "n_faces": d["n_faces"]}
    m = res["mixed"]
    out = {"metric": METRIC, "value": m["value"], "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 particle state/push/march, f64 barycentrics in flight, deposit+fields",
           "data": "synthetic",
           "config": {"workload": "tet_pair_plasma", "n_tets": nt, "n_edges": m["n_edges"],
                      "n_faces": m["n_faces"], "n_particles": n_p, "theta": w.extra["theta"],
                      "pusher": "boris", "precision": "mixed", "resort_every": resort,
                      "spai_level": 1},
           "roofline": m["roofline"], "stage_ms_per_step": m["stage_ms_per_step"],
           "gauss_rel": m["gauss_rel"], "divb_rel": m["divb_rel"],
           "pieces_per_particle_step": m["pieces_per_particle_step"]}
    if "fp64" in res:
        f = res["fp64"]
        out["fp64"] = {k: f[k] for k in ("value", "ms_per_step", "roofline", "stage_ms_per_step",
                                         "gauss_rel", "divb_rel")}
        out["mixed_vs_fp64"] = m["value"] / f["value"]
    del w
    if not args.no_cpu:
        log("timing the tetrahedral CPU oracle on a sample")
        out["cpu_baseline"] = tet_cpu_baseline(n_p)
    return out


def tet_cpu_baseline(n_full, sample_pairs=400_000, sample_steps=20):
    """The FP64 tetrahedral oracle on the same mesh with a bounded sample."""
    from oracle import tet as O3
    from paper_1707_04333_amd import inputs as I
    from paper_1707_04333_amd import inputs3 as J
    w = J.tet_pair_plasma(n_pairs=sample_pairs)
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = O3.OracleSim3(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=1,
                         b_ext=w.extra["b_ext"])
    osim.step(1)
    t0 = time.perf_counter()
    osim.step(sample_steps)
    el = time.perf_counter() - t0
    n = sum(s.n for s in osim.species)
    return {"value": n * sample_steps / el, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"same mesh ({w.mesh.n_tets} tetrahedra, FP64 field update), {n} of the "
                       f"{n_full} particles, {sample_steps} steps after 1 warm-up step, "
                       f"single-threaded FP64 C oracle; {el:.1f} s")}


def make_workload(name, args, precision):
    from paper_1707_04333_amd import inputs as I
    if name == "pair":
        return I.pair_plasma(n_pairs=args.pairs, theta=args.theta, precision=precision)
    if name == "large":
        return I.large_run(n_particles=args.large_particles, precision=precision)
    if name == "boosted":
        w = I.boosted_oscillator()
    elif name == "cyclotron":
        w = I.cyclotron()
    else:
        raise SystemExit(f"unknown workload {name}")
    w.precision = precision
    return w


def workload_config(name, w, info, pusher, resort, args):
    cfg = {"workload": w.name, "n_tris": info["n_tris"], "n_edges": info["n_edges"],
           "n_particles": w.n_particles, "pusher": pusher, "precision": "fp64",
           "resort_every": resort, "spai_level": w.spai_level}
    if name == "pair":
        cfg["theta"] = args.theta
    if name == "large":
        cfg.update({"grade": 10.0, "absorbing_layer": True, "theta": w.extra["theta"],
                    "beam_fraction": 0.05, "beam_gamma": 20.0})
    return cfg


def run_workload(name, args, pusher=None, resort=None):
    """FP64 (the value) and the two mixed forms of one workload."""
    w = make_workload(name, args, "fp64")
    pusher = pusher or args.pusher or ("boris" if name == "pair" else w.pusher)
    species_n = [s.n for s in w.species]
    n_p = w.n_particles
    counted = (name == "large" and args.large_particles == 128_000_000) or \
        (name == "pair" and args.pairs == DEFAULT_PAIRS)
    tfile = TRAFFIC_FILE if name == "large" else PAIR_TRAFFIC_FILE
    pin = (args.tile, args.scan, args.defer_exits)
    r64 = run_gpu(w, "fp64", args.steps, args.warmup, pusher, resort, pin)
    issue = counted and name == "large"
    rec = {"fp64": leg_record(r64, n_p, args.steps, species_n, False,
                              measured_traffic("fp64", tfile, tile=r64["tile"], scan=r64["scan"],
                                               defer=r64["defer"]) if counted else None,
                              measured_valu("fp64", tile=r64["tile"], scan=r64["scan"],
                                            defer=r64["defer"]) if issue else None)}
    if not args.no_mixed:
        for prec in ("mixed", "mixed_f64field"):
            r = run_gpu(w, prec, args.steps, args.warmup, pusher, resort or r64["resort"], pin)
            rec[prec] = leg_record(r, n_p, args.steps, species_n, True,
                                   measured_traffic(prec, tfile, tile=r["tile"], scan=r["scan"],
                                                    defer=r["defer"]) if counted else None,
                                   measured_valu(prec, tile=r["tile"], scan=r["scan"],
                                                 defer=r["defer"]) if issue else None)
            rec[prec]["vs_fp64"] = rec[prec]["value"] / rec["fp64"]["value"]
    cfg = workload_config(name, w, r64["info"], pusher, r64["resort"], args)
    return w, cfg, rec, r64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--theta", type=float, default=0.1)
    ap.add_argument("--pusher", default=None)
    ap.add_argument("--pairs", type=int, default=DEFAULT_PAIRS)
    ap.add_argument("--large-particles", type=int, default=128_000_000)
    ap.add_argument("--no-fp64", action="store_true", help="tetrahedral workload only")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-pair", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=None,
                    help="pin the particle tile (a multiple of 256 in 512..2048) after the "
                         "autotuner, e.g. to take counters at a fixed launch shape")
    ap.add_argument("--scan", type=int, default=None, help="pin the scan width (8, 16, 64)")
    ap.add_argument("--defer-exits", type=int, default=None, choices=(0, 1),
                    help="pin the FP32 legs' exit mode (FP64 always defers)")
    ap.add_argument("--batched-precision", default="mixed", choices=("mixed", "fp64"),
                    help="precision of --workload batched")
    ap.add_argument("--timing-overhead", action="store_true",
                    help="step time of the pair plasma with each stage-timing mode, in "
                         "windows separated by idle (for a kernel trace)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device with torch (a plain copy kernel "
                         "of known size, for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copied 1 GiB device-to-device")

    if args.timing_overhead:
        print(json.dumps(run_timing_overhead(args)))
        return
    if args.workload.startswith("synchro"):
        print(json.dumps(run_synchro(args)))
        return
    if args.workload == "bernstein":
        print(json.dumps(run_bernstein(args)))
        return
    if args.workload == "tet":
        print(json.dumps(run_tet(args)))
        return
    if args.workload == "batched":
        print(json.dumps(run_batched("boris", precision=args.batched_precision)))
        return
    name = args.workload
    log(f"generating workload {name}")
    resort = None
    if name == "large":
        resort = LARGE_RESORT
    elif args.no_autotune:
        resort = 20
    w, cfg, rec, r64 = run_workload(name, args, resort=resort)
    f64 = rec["fp64"]
    out = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": f64["roofline"],
        "valu_issue": f64["valu_issue"],
        "tuning": {"tile": f64["tile"], "scan_lanes": f64["scan_lanes"],
                   "defer_exits": f64["defer_exits"], "resort_every": f64["resort_every"]},
        "stage_ms_per_step": f64["stage_ms_per_step"],
        "gauss_rel": f64["gauss_rel"],
        "hbm_gbs_step": f64["hbm_gbs_step"],
        "sorts_in_timed_steps": f64["sorts_in_timed_steps"],
        "aligned_warmup_steps": r64["warmup_steps"],
    }
    for prec in ("mixed", "mixed_f64field"):
        if prec in rec:
            out[prec] = rec[prec]
    if "mixed" in rec:
        out["mixed_vs_fp64"] = rec["mixed"]["vs_fp64"]
    try:
        ceil = copy_ceiling_gbs()
        out["copy_ceiling_gbs"] = ceil
        out["roofline"]["frac_of_copy_ceiling"] = out["roofline"]["achieved"] / ceil
    except Exception as ex:  # the copy needs torch on the GPU
        log(f"copy ceiling not measured: {ex}")
    if name == "large" and not args.no_pair:
        log("pair plasma leg (199,712 triangles, 16M particles)")
        pargs = argparse.Namespace(**vars(args))
        _, pcfg, prec_rec, _ = run_workload("pair", pargs)
        out["pair_plasma"] = {"config": pcfg, **prec_rec}
    if not args.no_batched and name in ("large", "pair"):
        out["batched"] = run_batched("boris")
        out["batched_fp64"] = run_batched("boris", precision="fp64")
        out["batched"]["vs_fp64"] = out["batched"]["value"] / out["batched_fp64"]["value"]
    if not args.no_cpu and name in ("large", "pair"):
        log("timing the CPU oracle on the headline workload")
        out["cpu_baseline"] = cpu_baseline(w, cfg["pusher"])
    del w
    print(json.dumps(out))


if __name__ == "__main__":
    main()
