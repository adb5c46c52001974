"""O-PM: the long-range (particle-mesh) part of P3M, written out step by step.

The guide's PM part uses a PM_gridsize^3 periodic grid and FFTs (CONCEPT
User's Guide, Ch. 5 "Parameters", entries PM_gridsize and PM_scale; Ch. 3
lists FFTW for the transforms). It does not give the discretisation. The
readings taken here, each a standard choice:

1. Cloud-in-cell (CIC) mass assignment with nodes at c*h, h = L/N_g:
       rho(c) = h^-3 * sum_j m_j prod_d w(x_{j,d}/h - c_d),  w(t) = max(0, 1 - |t|)
   on periodic node indices (sum of rho h^3 = total mass).
2. rho_k = FFT(rho) (unnormalised forward transform, NumPy convention).
3. phi_k = G(k) rho_k with the Gaussian-split Green's function
       G(k) = -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^p),  G(0) = 0,
   k = 2 pi n / L with n_d in [-N_g/2, N_g/2) (the Nyquist index kept),
   W(k) = prod_d sinc^2(pi n_d / N_g) the CIC window, p = 2 (one power
   for assignment, one for interpolation; p = 0 switches deconvolution off).
   G(0) = 0 solves for rho minus its mean: the comoving neutralising
   background of periodic gravity.
4. phi = IFFT(phi_k) with the 1/N_g^3 normalisation.
5. Fourth-order central difference (order 2 also available):
       (D_d phi)(c) = [8 (phi(c+e_d) - phi(c-e_d)) - (phi(c+2e_d) - phi(c-2e_d))] / (12 h)
6. a_PM(x_i) = - sum_c prod_d w(x_{i,d}/h - c_d) (D phi)(c), the same CIC
   weights as the deposit (needed for zero self-force and momentum
   conservation).
"""
from __future__ import annotations

import numpy as np


def _as_mass(mass, n):
    if np.ndim(mass) == 0:
        return np.full(n, float(mass))
    return np.asarray(mass, dtype=np.float64)


def cic_weights(pos, box, ng):
    """Lower node index (3, N) and the fractional offset (3, N) of each particle."""
    h = box / ng
    t = np.asarray(pos, dtype=np.float64) / h
    i0 = np.floor(t)
    frac = t - i0
    i0 = np.mod(i0.astype(np.int64), ng)
    return i0, frac


def _corners(i0, frac, ng):
    """Yield (flat node index, weight) for the 8 CIC corners."""
    for a in (0, 1):
        ix = (i0[0] + a) % ng
        wx = frac[0] if a else 1.0 - frac[0]
        for b in (0, 1):
            iy = (i0[1] + b) % ng
            wy = frac[1] if b else 1.0 - frac[1]
            for c in (0, 1):
                iz = (i0[2] + c) % ng
                wz = frac[2] if c else 1.0 - frac[2]
                yield (ix * ng + iy) * ng + iz, wx * wy * wz


def cic_deposit(pos, mass, box, ng):
    """Mass density on the nodes, shape (ng, ng, ng)."""
    pos = np.asarray(pos, dtype=np.float64)
    m = _as_mass(mass, pos.shape[1])
    h = box / ng
    i0, frac = cic_weights(pos, box, ng)
    rho = np.zeros(ng ** 3)
    for flat, w in _corners(i0, frac, ng):
        rho += np.bincount(flat, weights=m * w, minlength=ng ** 3)
    return rho.reshape(ng, ng, ng) / h ** 3


def cic_interp(field, pos, box):
    """CIC interpolation of node fields (C, ng, ng, ng) to positions -> (C, N)."""
    field = np.asarray(field, dtype=np.float64)
    ng = field.shape[-1]
    flat_field = field.reshape(field.shape[0], -1)
    i0, frac = cic_weights(pos, box, ng)
    out = np.zeros((field.shape[0], np.asarray(pos).shape[1]))
    for flat, w in _corners(i0, frac, ng):
        out += w * flat_field[:, flat]
    return out


def wavenumbers(ng, box):
    """Integer wavenumbers n (x, y full; z half) and the squared k = 2 pi n / L."""
    n_full = np.fft.fftfreq(ng, d=1.0 / ng)
    n_half = np.fft.rfftfreq(ng, d=1.0 / ng)
    nx = n_full[:, None, None]
    ny = n_full[None, :, None]
    nz = n_half[None, None, :]
    kf = 2.0 * np.pi / box
    k2 = kf * kf * (nx * nx + ny * ny + nz * nz)
    return nx, ny, nz, k2


def green(ng, box, r_s, G=1.0, deconv_power=2):
    """Gaussian-split Green's function on the half-complex grid (ng, ng, ng//2+1)."""
    nx, ny, nz, k2 = wavenumbers(ng, box)
    W = (np.sinc(nx / ng) * np.sinc(ny / ng) * np.sinc(nz / ng)) ** 2
    k2safe = np.where(k2 == 0.0, 1.0, k2)
    g = -4.0 * np.pi * G * np.exp(-k2 * r_s * r_s) / (k2safe * W ** deconv_power)
    g[0, 0, 0] = 0.0
    return g


def potential(rho, box, r_s, G=1.0, deconv_power=2):
    """Long-range potential on the nodes from the node density."""
    ng = rho.shape[0]
    rho_k = np.fft.rfftn(rho)
    phi_k = green(ng, box, r_s, G, deconv_power) * rho_k
    return np.fft.irfftn(phi_k, s=rho.shape, axes=(0, 1, 2))


def fd_gradient(phi, box, order=4):
    """Central finite-difference gradient, shape (3, ng, ng, ng)."""
    ng = phi.shape[0]
    h = box / ng
    out = np.empty((3,) + phi.shape)
    for d in range(3):
        p1 = np.roll(phi, -1, axis=d)     # phi(c + e_d)
        m1 = np.roll(phi, 1, axis=d)      # phi(c - e_d)
        if order == 2:
            out[d] = (p1 - m1) / (2.0 * h)
        elif order == 4:
            p2 = np.roll(phi, -2, axis=d)
            m2 = np.roll(phi, 2, axis=d)
            out[d] = (8.0 * (p1 - m1) - (p2 - m2)) / (12.0 * h)
        else:
            raise ValueError("fd order must be 2 or 4")
    return out


def pm_accel(pos, mass, box, ng, r_s, G=1.0, fd_order=4, deconv_power=2,
             targets=None):
    """Long-range P3M acceleration, shape (3, T) for the target indices."""
    pos = np.asarray(pos, dtype=np.float64)
    rho = cic_deposit(pos, mass, box, ng)
    phi = potential(rho, box, r_s, G, deconv_power)
    grad = fd_gradient(phi, box, fd_order)
    where = pos if targets is None else pos[:, np.asarray(targets)]
    return -cic_interp(grad, where, box)
