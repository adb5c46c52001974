"""Background expansion and the comoving leapfrog coefficients (FP64 CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring). The guide sets the
background by H0, Omega_m, Omega_Lambda and a_begin and the time step as a
fraction of the age of the universe (CONCEPT User's Guide, Ch. 5); positions
and momenta are comoving (Ch. 6). With canonical momenta p = a^2 m dx/dt:

    H(a)     = H0 sqrt(Omega_m a^-3 + (1 - Omega_m - Omega_Lambda) a^-2 + Omega_Lambda)
    t(a)     = int_0^a da / (a H)
    c_kick   = int dt / a   = int_{a0}^{a1} da / (a^2 H)
    c_drift  = int dt / a^2 = int_{a0}^{a1} da / (a^3 H)

Evaluated with scipy's adaptive quadrature (QUADPACK) and Brent's root
finder; nothing here is shared with the library's own quadrature.
"""
from __future__ import annotations

import math

from scipy import integrate, optimize


def hubble(a, H0, Om, OL):
    Ok = 1.0 - Om - OL
    return H0 * math.sqrt(Om / a ** 3 + Ok / a ** 2 + OL)


def age(a, H0, Om, OL):
    val, _ = integrate.quad(lambda x: 1.0 / (x * hubble(x, H0, Om, OL)), 0.0, a,
                            epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def scale_factor(t, H0, Om, OL):
    # bracket the root by doubling and halving (t(a) increases from 0)
    hi = 1.0
    while age(hi, H0, Om, OL) < t:
        hi *= 2.0
    lo = hi
    while age(lo, H0, Om, OL) > t:
        lo *= 0.5
    if lo == hi:
        return hi
    return optimize.brentq(lambda a: age(a, H0, Om, OL) - t, lo, hi,
                           xtol=1e-300, rtol=1e-15, maxiter=500)


def kick_drift(a0, a1, H0, Om, OL):
    ck, _ = integrate.quad(lambda x: 1.0 / (x * x * hubble(x, H0, Om, OL)), a0, a1,
                           epsabs=0.0, epsrel=1e-13, limit=400)
    cd, _ = integrate.quad(lambda x: 1.0 / (x ** 3 * hubble(x, H0, Om, OL)), a0, a1,
                           epsabs=0.0, epsrel=1e-13, limit=400)
    return ck, cd
