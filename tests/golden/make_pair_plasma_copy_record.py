"""Writes tests/golden/pair_plasma_copy_theta0.1.npz: the oracle's record of
the 1/16-area copy of the relativistic pair-plasma Bernstein workload
(Sec. III.C; 0.125 m doubly periodic square, 79 x 79 cells, 12,482
triangles, 500,000 electron-positron pairs, theta = kT/(m c^2) = 0.1,
B0 = 1 T, omega_c/omega_p = 2, dt = 0.2/omega_c, Boris pusher), 1000 steps
in the oracle's single-threaded parity mode:

* ex: E_x (float32) at 79 points on the line y = L/2, x = (i + 1/2) L/79,
  after every step (the oracle's Whitney gather, Sec. II.B);
* we, wb, wk: electric, magnetic and kinetic energy after every step;
* gauss: the largest Gauss-law residual over the free nodes at the end,
  relative to the largest nodal charge.

Run from the repository root:  python tests/golden/make_pair_plasma_copy_record.py
(about 15 minutes of one core)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1707_04333_amd import inputs as I  # noqa: E402

THETA, STEPS, NX = 0.1, 1000, 79
OUT = os.path.join(ROOT, "tests", "golden", "pair_plasma_copy_theta0.1.npz")


def probe_points(length, nx):
    return np.stack([(np.arange(nx) + 0.5) * length / nx, np.full(nx, 0.5 * length)], axis=1)


def main():
    w = I.pair_plasma_small(theta=THETA, precision="fp64")
    length = 0.125
    sp = [(s.q, s.m, s.w, s.tri, s.lam, s.u) for s in w.species]
    osim = O.OracleSim(w.mesh, w.dt, sp, I.EPS0, I.MU0, I.C_LIGHT, spai_level=w.spai_level,
                       bz_ext=w.bz_ext)
    tri, lam = I.locate_points(w.mesh, probe_points(length, NX))
    bary = np.stack([(1.0 - lam[:, 0]) - lam[:, 1], lam[:, 0], lam[:, 1]], axis=1)
    ex = np.zeros((STEPS, NX), np.float32)
    en = np.zeros((STEPS, 3))
    q0, d0 = osim.charge(), osim.d.copy()
    t0 = time.time()
    for n in range(STEPS):
        osim.step(1, w.pusher)
        ex[n] = [O.gather_e(osim, tri[i], bary[i])[0] for i in range(NX)]
        en[n] = osim.energies()
        if n % 50 == 0:
            print(f"step {n} {time.time() - t0:.0f} s W_E {en[n, 0]:.4g}", flush=True)
    free = osim.T.node_free.astype(bool)
    res = osim.T.divergence(osim.d - d0) - (osim.charge() - q0)
    qmax = max(np.abs(q0).max(), np.abs(osim.charge()).max())
    gauss = float(np.abs(res[free]).max() / qmax)
    np.savez(OUT, ex=ex, we=en[:, 0], wb=en[:, 1], wk=en[:, 2], gauss=gauss,
             dt=w.dt, omega_c=w.extra["omega_c"], theta=THETA, length=length,
             lost=osim.lost)
    print("wrote", OUT, "gauss", gauss)


if __name__ == "__main__":
    main()
