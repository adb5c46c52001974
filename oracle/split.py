"""The Gaussian long/short force split.

The guide splits gravity at a scale r_s (PM_scale, in PM cells) into a
long-range part solved on the mesh and a short-range part summed over pairs
closer than a cutoff r_c (P3M_cutoff, in units of r_s); by its Ch. 5, cutting
off at 4.8 r_s or beyond drops under one percent of the force (CONCEPT User's
Guide, Ch. 5 "Parameters", entries PM_scale and P3M_cutoff). The functional form is not given; the reading taken here is
the Gaussian split, the one common convention that matches that statement:

    long range:  potential kernel  exp(-k^2 r_s^2) / k^2     (Fourier space)
    short range: pair force Newton * f(r),
                 f(r) = erfc(r / (2 r_s)) + r / (r_s sqrt(pi)) * exp(-r^2 / (4 r_s^2))

f(0) = 1 and f decreases monotonically to 0; with u = r/(2 r_s),
f = erfc(u) + (2u/sqrt(pi)) exp(-u^2). The fraction of a pair's force left
out at the cutoff is f(r_c): f(4.8 r_s) = 0.0092 < 1 % < f(4.75 r_s) = 0.0103.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc

SQRT_PI = np.sqrt(np.pi)


def split_factor(r, r_s):
    """Short-range share f(r) of the Newtonian pair force (float64)."""
    r = np.asarray(r, dtype=np.float64)
    u = r / (2.0 * r_s)
    return erfc(u) + (2.0 / SQRT_PI) * u * np.exp(-u * u)
