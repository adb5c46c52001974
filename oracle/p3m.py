"""O-P3M: short-range pair sum plus particle-mesh long range.

P3M as the guide names it (CONCEPT User's Guide, Ch. 1 and Ch. 5: gravity by
PP, PM or P3M; the split at PM_scale and the cutoff P3M_cutoff): the total
acceleration is the sum of ``pp.pp_accel`` and ``pm.pm_accel`` with the same
r_s, and the force on a particle is its mass times that acceleration. This is
the parity reference for the GPU force path.
"""
from __future__ import annotations

import numpy as np

from .pm import pm_accel
from .pp import pp_accel


def params_from_cells(box, ng, rs_cells, cutoff_rs):
    """r_s = rs_cells * h and r_c = cutoff_rs * r_s (guide Ch. 5 units)."""
    h = box / ng
    r_s = rs_cells * h
    return r_s, cutoff_rs * r_s


def p3m_accel(pos, mass, box, ng, rs_cells=1.25, cutoff_rs=4.5, eps=0.0, G=1.0,
              fd_order=4, deconv_power=2, targets=None, pp_method="auto"):
    r_s, r_c = params_from_cells(box, ng, rs_cells, cutoff_rs)
    a_pp = pp_accel(pos, mass, box, r_s, r_c, eps, G, targets=targets,
                    method=pp_method)
    a_pm = pm_accel(pos, mass, box, ng, r_s, G, fd_order, deconv_power,
                    targets=targets)
    return a_pp + a_pm


def _target_mass(mass, n, targets):
    if np.ndim(mass) == 0:
        return float(mass)
    m = np.asarray(mass, dtype=np.float64)
    return m if targets is None else m[np.asarray(targets)]


def p3m_force(pos, mass, box, ng, rs_cells=1.25, cutoff_rs=4.5, eps=0.0, G=1.0,
              fd_order=4, deconv_power=2, targets=None, pp_method="auto"):
    """F_i = m_i * (a_PP + a_PM), shape (3, T)."""
    a = p3m_accel(pos, mass, box, ng, rs_cells, cutoff_rs, eps, G, fd_order,
                  deconv_power, targets, pp_method)
    return a * _target_mass(mass, np.shape(pos)[1], targets)


def pp_force(pos, mass, box, ng, rs_cells=1.25, cutoff_rs=4.5, eps=0.0, G=1.0,
             targets=None, pp_method="auto"):
    r_s, r_c = params_from_cells(box, ng, rs_cells, cutoff_rs)
    a = pp_accel(pos, mass, box, r_s, r_c, eps, G, targets=targets, method=pp_method)
    return a * _target_mass(mass, np.shape(pos)[1], targets)


def pm_force(pos, mass, box, ng, rs_cells=1.25, G=1.0, fd_order=4, deconv_power=2,
             targets=None):
    r_s = rs_cells * box / ng
    a = pm_accel(pos, mass, box, ng, r_s, G, fd_order, deconv_power, targets=targets)
    return a * _target_mass(mass, np.shape(pos)[1], targets)
