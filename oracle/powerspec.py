"""Power spectrum of the particle density on the PM grid, and sigma(R).

The guide reduces snapshots to power spectra computed on the PM grid
(CONCEPT User's Guide, Ch. 5: PM_gridsize is also the power-spectrum grid;
R_tophat sets the radius of the top-hat for sigma, the rms density
variation; Ch. 8 powerspec test: sigma from the spectrum against the rms of
particle counts in cubes). It gives no estimator; the readings written out
here:

1. Density contrast on the nodes from the CIC deposit of ``pm``:
   delta(c) = rho(c) / rho_bar - 1, rho_bar = total mass / L^3.
2. delta_k = FFT(delta) (unnormalised), P(k) = L^3 |delta_k|^2 / N_g^6, for
   k != 0, divided by W(k)^2 (W = prod_d sinc^2(pi n_d / N_g), the CIC window)
   unless deconvolution is off.
3. Shells of unit width in |n| (k = 2 pi n / L): bin b holds the modes with
   b + 1/2 <= |n| < b + 3/2, b = 0 .. nbins - 1; P_b and k_b are averages over
   the bin's modes of the full k-space (each half-spectrum entry with
   0 < n_z < N_g/2 stands for two modes), modes_b their number.
4. sigma^2(R) = (1 / L^3) sum_{k != 0} P(k) W_TH(k R)^2 over every grid mode,
   W_TH(x) = 3 (sin x - x cos x) / x^3: the variance of the density contrast
   smoothed with a sphere of radius R, as a sum over the grid's own modes
   (R = 0 gives the grid variance of delta, by Parseval).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .pm import cic_deposit


def tophat_window(x):
    """W_TH(x) = 3 (sin x - x cos x) / x^3, with W_TH(0) = 1."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, full)


def _modes(ng):
    """Integer wavenumbers (x, y full; z half) and the full-space multiplicity."""
    n_full = np.fft.fftfreq(ng, d=1.0 / ng)
    n_half = np.fft.rfftfreq(ng, d=1.0 / ng)
    nx, ny, nz = np.meshgrid(n_full, n_full, n_half, indexing="ij")
    mult = np.where((nz == 0) | (nz == ng // 2), 1.0, 2.0)
    return nx, ny, nz, mult


def power_spectrum(pos, mass, box, ng, nbins, deconvolve=True, r_tophat=0.0):
    """(k_b, P_b, modes_b, sigma(r_tophat)) of the particle density."""
    pos = np.asarray(pos, dtype=np.float64)
    rho = cic_deposit(pos, mass, box, ng)
    total = np.sum(rho) * (box / ng) ** 3
    rho_bar = total / box ** 3
    delta = rho / rho_bar - 1.0
    dk = np.fft.rfftn(delta)
    nx, ny, nz, mult = _modes(ng)
    p = box ** 3 * np.abs(dk) ** 2 / float(ng) ** 6
    if deconvolve:
        W = (np.sinc(nx / ng) * np.sinc(ny / ng) * np.sinc(nz / ng)) ** 2
        p = p / W ** 2
    nabs = np.sqrt(nx * nx + ny * ny + nz * nz)
    nonzero = nabs > 0
    b = np.floor(nabs - 0.5).astype(np.int64)
    sel = nonzero & (b >= 0) & (b < nbins)
    modes = np.bincount(b[sel], weights=mult[sel], minlength=nbins)
    psum = np.bincount(b[sel], weights=(mult * p)[sel], minlength=nbins)
    ksum = np.bincount(b[sel], weights=(mult * nabs)[sel], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        P = np.where(modes > 0, psum / modes, 0.0)
        k = np.where(modes > 0, 2.0 * np.pi / box * ksum / modes, 0.0)
    kr = 2.0 * np.pi / box * nabs * r_tophat
    s2 = np.sum((mult * p * tophat_window(kr) ** 2)[nonzero]) / box ** 3
    return k, P, modes, float(np.sqrt(s2))


def cic_shot_noise_factor(ng):
    """prod_d (1 - (2/3) sin^2(pi n_d / N_g)) on the half-spectrum modes: the sum
    over aliases of the squared CIC window, which multiplies the Poisson
    noise L^3 / N of a spectrum measured without deconvolution."""
    nx, ny, nz, _ = _modes(ng)
    f = 1.0
    for n in (nx, ny, nz):
        f = f * (1.0 - (2.0 / 3.0) * np.sin(np.pi * n / ng) ** 2)
    return f
