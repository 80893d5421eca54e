"""Experiment drivers on the library: the synchrocyclotron of Sec. III.A.

The accelerating gap carries an applied RF field E = (E0 sin(phase), 0)
inside a vertical strip.  It is given to the library as edge DoFs (the
line integral E0 (x_hi - x_lo) on every edge whose midpoint lies in the
strip) whose amplitude the driver sets before each step
(fetd_set_ext_scale); the phase advances by 2 pi f dt with f the constant
non-relativistic cyclotron frequency f0 = eB/(2 pi m) or, synchronised,
f0/gamma of the electron (Sec. III.A: f = qB/(2 pi gamma m0)).
"""
from __future__ import annotations

import math

import numpy as np

from . import fetdpic as fp


def gap_field(node_xy: np.ndarray, edges: np.ndarray, e0: float, gap_x: float,
              gap: float) -> np.ndarray:
    """Edge DoFs of the uniform field (e0, 0) restricted to the strip
    |x - gap_x| < gap/2: e0 (x_hi - x_lo) on edges (lo, hi) whose midpoint
    lies in the strip, zero elsewhere."""
    xl = node_xy[edges[:, 0], 0]
    xh = node_xy[edges[:, 1], 0]
    mid = 0.5 * (xl + xh)
    return np.where(np.abs(mid - gap_x) < 0.5 * gap, e0 * (xh - xl), 0.0)


class RFDrive:
    """Phase of the gap field: sin(phase) is the amplitude of the step about
    to run; advance() moves the phase by 2 pi f dt."""

    def __init__(self, f0: float, dt: float, synchronised: bool):
        self.f0, self.dt, self.sync = f0, dt, synchronised
        self.phase = 0.0

    def amplitude(self) -> float:
        return math.sin(self.phase)

    def advance(self, gamma: float) -> None:
        f = self.f0 / gamma if self.sync else self.f0
        self.phase += 2.0 * math.pi * f * self.dt


def run_synchrocyclotron(w, steps: int, pusher: str = "boris_tan", device: int = 0,
                         record_every: int = 1):
    """Run a synchrocyclotron workload (inputs.synchrocyclotron) on the GPU.
    Returns per recorded step: step, gamma, kinetic energy [J], position
    (x, y) of the electron; and at the end the diagnostics, the particle
    state and the edge field e."""
    from . import inputs as I
    sim = fp.from_workload(w, device=device)
    edges = sim.field("edges").reshape(-1, 2)
    x = w.extra
    sim.fields_set(bz_ext=x["bz_tri"],
                   e_ext=gap_field(w.mesh.node_xy, edges, x["e0"], x["gap_x"], x["gap"]))
    c = x.get("c", I.C_LIGHT)
    drive = RFDrive(x["f0"], w.dt, x["case"] == "synched")
    sp = w.species[0]
    rec = {"step": [], "gamma": [], "ekin": [], "xy": []}
    vxy = w.mesh.vertex_xy()
    for n in range(steps + 1):
        p = sim.particles(0)
        if p["u"].shape[0] == 0:
            break
        u = p["u"][0]
        gamma = math.sqrt(1.0 + (u @ u) / (c * c))
        if n % record_every == 0 or n == steps:
            L = np.empty(3)
            r = int(p["slot"][0])
            L[(r + 1) % 3], L[(r + 2) % 3] = p["lam"][0]
            L[r] = (1.0 - p["lam"][0][0]) - p["lam"][0][1]
            rec["step"].append(n)
            rec["gamma"].append(gamma)
            # kinetic energy (gamma - 1) m c^2 with the rest mass of the species
            rec["ekin"].append((gamma - 1.0) * sp.m * c * c if x["case"] != "nonrel"
                               else 0.5 * sp.m * float(u @ u))
            rec["xy"].append(L @ vxy[int(p["tri"][0])])
        if n == steps:
            break
        sim.set_ext_scale(drive.amplitude())
        sim.step(1, pusher)
        drive.advance(gamma)
    out = {k: np.asarray(v) for k, v in rec.items()}
    out["diag"] = sim.diagnostics()
    out["particles"] = sim.particles(0)
    out["e"] = sim.field("e")
    sim.close()
    return out
