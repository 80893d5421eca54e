"""Benchmark: particle-steps/s of the full PIC step on one MI355X.

Workload: relativistic pair-plasma Bernstein configuration — doubly
periodic 0.5 m x 0.5 m mesh of 199,712 triangles (316 x 316 torus),
8M electrons + 8M positrons in collocated pairs, in-plane
Maxwell-Juttner momenta (kT/mc^2 = theta), uniform B0 = 1 T with
omega_c/omega_p = 2, dt = 0.2/omega_c, mixed precision (FP32 positions,
momenta, gather/push/track; FP64 deposit, field update and Gauss
accounting), particles re-sorted by triangle every 20 steps.

A step is one pass of the whole path: Faraday + gather record, the fused
gather/push/track/deposit stage for both species, Ampere, the SPAI SpMV,
and (every 20th step) the counting sort.  The same workload in FP64 is
timed beside it, the Gauss residual is reported for both, the fused
particle kernel is placed on the HBM roofline from HIP-event timings of
its launches inside the timed region, and the FP64 CPU oracle is timed on
a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-steps/sec + achieved HBM GB/s; mixed/batched vs FP64 at Gauss residual")
HBM_PEAK_GBS = 8000.0


def particle_launch_bytes(n_particles, nf, ne, fp32):
    """Algorithmic bytes of one fused particle-stage launch: every particle
    reads and writes its state (key 4 B, barycentric pair and momentum
    2 x 2 reals), every triangle's record (8 reals), gradients (6 reals,
    padded to 8 in FP32), edge and neighbour tables (16 B each) are read
    once, and every edge's FP64 current is read and written once."""
    r = 4 if fp32 else 8
    per_particle = 2 * (4 + 4 * r)
    per_tri = 8 * r + (8 if fp32 else 6) * r + 16 + 16
    return n_particles * per_particle + nf * per_tri + ne * 16


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(w, precision, steps, warmup, pusher):
    from paper_1707_04333_amd import fetdpic as fp
    log(f"{precision}: creating simulation ({w.n_particles} particles)")
    sim = fp.from_workload(w, precision=precision, spai_level=w.spai_level, device=0)
    info = sim.info()
    sim.diagnostics()  # Gauss baseline at step 0
    sim.step(warmup, pusher)
    sim.sync()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(steps, pusher)
    sim.sync()
    t1 = time.perf_counter()
    stages = sim.stage_times()
    sim.profile(False)
    diag = sim.diagnostics()
    sim.close()
    log(f"{precision}: {steps} steps in {t1 - t0:.3f} s")
    return dict(elapsed=t1 - t0, stages=stages, diag=diag, info=info)


def cpu_baseline(w_full, pusher, sample_pairs=500_000, sample_steps=25):
    import oracle
    from paper_1707_04333_amd import inputs as I
    w = I.pair_plasma(n_pairs=sample_pairs, theta=w_full.extra["theta"], precision="fp64")
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = oracle.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT,
                            spai_level=w.spai_level, bz_ext=w.bz_ext)
    osim.step(1, pusher)
    t0 = time.perf_counter()
    osim.step(sample_steps, pusher)
    el = time.perf_counter() - t0
    n = sum(s.n for s in osim.species)
    return {"value": n * sample_steps / el, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"same mesh ({w.mesh.n_tris} triangles, FP64 field update), "
                       f"{n} of the {w_full.n_particles} particles, {sample_steps} steps "
                       f"after 1 warm-up step, single-threaded FP64 C oracle; "
                       f"{el:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--theta", type=float, default=0.1)
    ap.add_argument("--pusher", default="boris")
    ap.add_argument("--pairs", type=int, default=8_000_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device with torch (a plain copy kernel "
                         "of known size, for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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
    from paper_1707_04333_amd import inputs as I
    log("generating workload")
    w = I.pair_plasma(n_pairs=args.pairs, theta=args.theta, precision="mixed")
    n_p = w.n_particles
    mixed = run_gpu(w, "mixed", args.steps, args.warmup, args.pusher)
    value = n_p * args.steps / mixed["elapsed"]
    info = mixed["info"]
    ms, launches = mixed["stages"]["particles"]
    per_launch_bytes = np.mean([particle_launch_bytes(s.n, info["n_tris"], info["n_edges"], True)
                                for s in w.species])
    avg_s = ms / 1e3 / max(launches, 1)
    achieved = per_launch_bytes / avg_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 particle state/push/track, f64 deposit+fields",
        "data": "synthetic",
        "config": {"workload": "pair_plasma_bernstein", "n_tris": info["n_tris"],
                   "n_edges": info["n_edges"], "n_particles": n_p, "theta": args.theta,
                   "pusher": args.pusher, "precision": "mixed", "resort_every": 20,
                   "spai_level": w.spai_level, "dt": w.dt},
        "roofline": {"bound": "hbm", "kernel": "k_particle_step", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_ms": avg_s * 1e3,
                     "algorithmic_bytes_per_launch": per_launch_bytes},
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in mixed["stages"].items()},
        "gauss_rel": mixed["diag"]["gauss_rel"],
        "hbm_gbs_step": None,
    }
    # whole-step effective bandwidth (particle stage + field stages)
    step_bytes = sum(particle_launch_bytes(s.n, info["n_tris"], info["n_edges"], True)
                     for s in w.species)
    out["hbm_gbs_step"] = step_bytes / (mixed["elapsed"] / args.steps) / 1e9
    if not args.no_fp64:
        w64 = I.pair_plasma(n_pairs=args.pairs, theta=args.theta, precision="fp64")
        r64 = run_gpu(w64, "fp64", args.steps, args.warmup, args.pusher)
        ms64, l64 = r64["stages"]["particles"]
        b64 = np.mean([particle_launch_bytes(s.n, info["n_tris"], info["n_edges"], False)
                       for s in w64.species])
        a64 = b64 / (ms64 / 1e3 / max(l64, 1)) / 1e9
        out["fp64"] = {"value": n_p * args.steps / r64["elapsed"],
                       "ms_per_step": r64["elapsed"] / args.steps * 1e3,
                       "gauss_rel": r64["diag"]["gauss_rel"],
                       "particle_kernel_gbs": a64, "particle_kernel_frac": a64 / HBM_PEAK_GBS,
                       "stage_ms_per_step": {k: v[0] / args.steps
                                             for k, v in r64["stages"].items()}}
        out["mixed_vs_fp64"] = value / out["fp64"]["value"]
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, args.pusher)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
