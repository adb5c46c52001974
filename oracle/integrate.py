"""Kick and drift, the two particle updates of the guide's time stepping.

The guide advances comoving positions and momenta (CONCEPT User's Guide,
Ch. 6: momenta in units of length*mass/time) with "kick" and "drift"
operations (Ch. 5 entry kick_algorithms; Ch. 8 tests drift and
kick_PP_with_Ewald) over one global time step (Ch. 5 entry Delta t_factor).
The guide gives no equations; with the time integrals folded into one
coefficient each (c_k, c_d; for a static background c_k = dt/2 in a
kick-drift-kick step and c_d = dt), the updates read:

    kick:   p <- p + c_k F
    drift:  x <- wrap(x + c_d (p / m)),  wrap(y) = y - L floor(y / L),
            with a result equal to L mapped to 0

Each product, quotient and sum is one IEEE double operation in exactly this
order (no fused multiply-add), so the results are reproducible bit for bit.
"""
from __future__ import annotations

import numpy as np


def kick(mom, force, c_kick):
    mom = np.asarray(mom, dtype=np.float64)
    f = np.asarray(force).astype(np.float64)
    return mom + c_kick * f


def wrap(y, box):
    y = np.asarray(y, dtype=np.float64)
    w = y - box * np.floor(y / box)
    return np.where(w >= box, 0.0, w)


def drift(pos, mom, mass, c_drift, box):
    pos = np.asarray(pos, dtype=np.float64)
    mom = np.asarray(mom, dtype=np.float64)
    m = float(mass) if np.ndim(mass) == 0 else np.asarray(mass, dtype=np.float64)[None, :]
    v = mom / m
    return wrap(pos + c_drift * v, box)


def kdk_step(pos, mom, mass, force_fn, dt, box, force=None):
    """One kick-drift-kick step with a static background; returns (pos, mom, force).

    ``force_fn(pos) -> (3, N)``; ``force`` is the force at the incoming
    positions if already known."""
    if force is None:
        force = force_fn(pos)
    mom = kick(mom, force, 0.5 * dt)
    pos = drift(pos, mom, mass, dt, box)
    force = force_fn(pos)
    mom = kick(mom, force, 0.5 * dt)
    return pos, mom, force
