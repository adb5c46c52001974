"""Writes the FP64 CPU reference gradient of the clustered differentiable
leapfrog at 16^3 particles (the 128^3 Plummer-mix workload's recipe on a
16^3 grid, 50 kick-drift-kick steps from rest), computed with the oracle
only: oracle.adjoint.leapfrog for the trajectory (oracle.p3m forces) and
oracle.adjoint.leapfrog_vjp with oracle.adjoint.p3m_vjp for its transpose.

Loss: the sum of squared final displacements (minimum image, from the
initial positions); the gradient is with respect to the initial positions.
Also recorded: the tangent-norm growth of the trajectory, |x_T(x0 + e v) -
x_T(x0)| / e for a seeded random unit direction v (e = 1e-7 of the box), and
the relative change of the gradient itself when x0 moves by 1e-12 of the box
along v (how well conditioned the gradient is).

Run from the repository root:  python tests/golden/make_plummer16_kdk_gradient.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint  # noqa: E402
from oracle import p3m as o_p3m  # noqa: E402
from paper_1510_07621_amd import ics  # noqa: E402

N_SIDE, GRID, STEPS, SEED = 16, 16, 50, 5
RS_CELLS, CUTOFF_RS, SOFT = 1.25, 4.5, 0.03


def main():
    n = N_SIDE ** 3
    pos = ics.plummer_mix(n, 1.0, seed=SEED)
    m = 1.0 / n
    eps = SOFT / N_SIDE
    force = lambda x: m * o_p3m.p3m_accel(x, m, 1.0, GRID, RS_CELLS, CUTOFF_RS, eps)
    vjp = lambda x, lam: adjoint.p3m_vjp(x, m, 1.0, GRID, lam, RS_CELLS, CUTOFF_RS, eps)
    for dt in (0.001, 0.01):
        xs, _ = adjoint.leapfrog(pos, np.zeros_like(pos), m, force, dt, 1.0, STEPS)
        s = xs[-1] - pos
        s -= np.round(s)
        loss = float(np.sum(s * s))
        x0b, _ = adjoint.leapfrog_vjp(xs, m, vjp, dt, 2.0 * s, np.zeros_like(pos))
        grad = x0b - 2.0 * s
        v = np.random.default_rng(7).normal(size=pos.shape)
        v /= np.linalg.norm(v)
        e = 1e-7
        xp, _ = adjoint.leapfrog(np.mod(pos + e * v, 1.0), np.zeros_like(pos), m, force, dt,
                                 1.0, STEPS)
        d = xp[-1] - xs[-1]
        d -= np.round(d)
        growth = float(np.linalg.norm(d) / e)
        # conditioning of the gradient itself: the same computation from
        # initial positions moved by 1e-12 of the box along v
        x1 = np.mod(pos + 1e-12 * v, 1.0)
        xs1, _ = adjoint.leapfrog(x1, np.zeros_like(pos), m, force, dt, 1.0, STEPS)
        s1 = xs1[-1] - x1
        s1 -= np.round(s1)
        x1b, _ = adjoint.leapfrog_vjp(xs1, m, vjp, dt, 2.0 * s1, np.zeros_like(pos))
        grad1 = x1b - 2.0 * s1
        cond = float(np.linalg.norm(grad1 - grad) / np.linalg.norm(grad))
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                            f"plummer16_kdk_grad_dt{dt:g}.txt")
        header = "\n".join([
            "FP64 CPU oracle gradient dL/dx0 (3 columns: x, y, z; one row per particle),",
            f"Plummer mix (70 % in 2000 spheres, 30 % uniform) of {n} particles, seed {SEED},",
            f"grid {GRID}^3, r_s = {RS_CELLS} cells, r_c = {CUTOFF_RS} r_s, eps = {SOFT} spacing, "
            f"G = 1, m = 1/N, {STEPS} KDK steps of dt = {dt:g} from rest;",
            "L = sum of squared final displacements (minimum image).",
            "Written by tests/golden/make_plummer16_kdk_gradient.py (oracle only).",
            f"loss {loss:.17g}",
            f"tangent_norm_growth {growth:.6g}",
            f"grad_change_at_1e-12 {cond:.6g}",
        ])
        np.savetxt(path, grad.T, fmt="%.10e", header=header)
        print(path, "loss", loss, "growth", growth, "grad change", cond, flush=True)


if __name__ == "__main__":
    main()
