"""O-EW: periodic gravity by direct Ewald summation, the accuracy truth.

The guide computes PP gravity with periodic images by Ewald summation
(CONCEPT User's Guide, Ch. 5 "Parameters", entries use_Ewald and
ewald_gridsize; Ch. 8 test kick_PP_with_Ewald). Here the sum is done
directly, with no table: for a source j seen from i, r = x_i - x_j and
r_n = r + n L,

    a_i = -G sum_j m_j [ sum_n r_n g(|r_n|)
                         + (4 pi / L^3) sum_{k != 0} (k / k^2) exp(-k^2/(4 alpha^2)) sin(k . r) ]
    g(s) = (erfc(alpha s) + (2 alpha s / sqrt(pi)) exp(-alpha^2 s^2)) / s^3

with the (j = i, n = 0) real-space term left out. This is the field of
point masses and all their periodic images in a neutralising uniform
background; it does not depend on alpha, which only moves work between the
two sums (truncated here far below double-precision rounding).

Softening (a stated reading; the guide gives only the Plummer radius,
Ch. 5 entry softeningfactors): the minimum-image partner's Newtonian term
r/|r|^3 is replaced by the Plummer term r/(|r|^2 + eps^2)^(3/2); all other
images stay Newtonian. This keeps the result alpha-independent.

The k-space sum is taken over a half space with structure factors
S(k) = sum_j m_j exp(i k . x_j), so its cost is O(N N_k).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

_SQRT_PI = math.sqrt(math.pi)
_KSPACE_EXPONENT = 40.0   # keep exp(-k^2/(4 alpha^2)) > e^-40
_REAL_SPAN = 7.0          # keep erfc(alpha s) down to erfc(7) ~ 4e-23


def _as_mass(mass, n):
    if np.ndim(mass) == 0:
        return np.full(n, float(mass))
    return np.asarray(mass, dtype=np.float64)


def _half_space_vectors(nk):
    r = np.arange(-nk, nk + 1)
    NX, NY, NZ = np.meshgrid(r, r, r, indexing="ij")
    n = np.stack([NX.ravel(), NY.ravel(), NZ.ravel()], axis=1)
    n2 = np.einsum("kd,kd->k", n, n)
    upper = (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | \
            ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))
    return n[upper & (n2 <= nk * nk) & (n2 > 0)]


def _phases(x, box, nk):
    """exp(i 2 pi n x_d / L) for n in [-nk, nk], each shape (2nk+1, len(x))."""
    n = np.arange(-nk, nk + 1)[:, None]
    return [np.exp(1j * (2.0 * np.pi / box) * n * x[:, d][None, :]) for d in range(3)]


def kspace_accel(pos, mass, box, alpha, G=1.0, targets=None, kchunk=256):
    """The Fourier-space part of the Ewald acceleration, shape (3, T)."""
    x = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)
    n = x.shape[0]
    m = _as_mass(mass, n)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    nk = int(math.ceil(math.sqrt(_KSPACE_EXPONENT) * alpha * box / math.pi))
    vecs = _half_space_vectors(nk)
    src = _phases(x, box, nk)
    dst = _phases(x[targets], box, nk)
    out = np.zeros((len(targets), 3))
    kf = 2.0 * np.pi / box
    for s in range(0, len(vecs), kchunk):
        v = vecs[s:s + kchunk]
        ix, iy, iz = (v[:, 0] + nk, v[:, 1] + nk, v[:, 2] + nk)
        S = (src[0][ix] * src[1][iy] * src[2][iz]) @ m            # (K,)
        e_t = dst[0][ix] * dst[1][iy] * dst[2][iz]                 # (K, T)
        k = kf * v
        k2 = np.einsum("kd,kd->k", k, k)
        coef = np.exp(-k2 / (4.0 * alpha * alpha)) / k2
        # half space: the -k term equals the +k term, hence the factor 2
        im = np.imag(e_t * np.conj(S)[:, None])                    # (K, T)
        out += 2.0 * (im * coef[:, None]).T @ k
    return -G * (4.0 * np.pi / box ** 3) * out.T


def realspace_accel(pos, mass, box, alpha, G=1.0, eps=0.0, targets=None, chunk=None):
    """The real-space part (with the softened minimum-image term), shape (3, T)."""
    x = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)
    n = x.shape[0]
    m = _as_mass(mass, n)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    r_max = _REAL_SPAN / alpha
    n_img = max(0, int(math.ceil(r_max / box - 0.5)))
    shifts = np.arange(-n_img, n_img + 1) * box
    out = np.zeros((len(targets), 3))
    step = chunk or max(1, 1_000_000 // max(n, 1))
    for s in range(0, len(targets), step):
        t = targets[s:s + step]
        d0 = x[t][:, None, :] - x[None, :, :]
        d0 -= box * np.round(d0 / box)
        self_mask = t[:, None] == np.arange(n)[None, :]
        acc = np.zeros((len(t), 3))
        for sx in shifts:
            for sy in shifts:
                for sz in shifts:
                    d = d0 + np.array([sx, sy, sz])
                    s2 = np.einsum("tjd,tjd->tj", d, d)
                    keep = s2 < r_max * r_max
                    if sx == 0 and sy == 0 and sz == 0:
                        keep &= ~self_mask & (s2 > 0.0)
                    sv = np.sqrt(np.where(keep, s2, 1.0))
                    g = (erfc(alpha * sv) + (2.0 * alpha / _SQRT_PI) * sv *
                         np.exp(-(alpha * sv) ** 2)) / sv ** 3
                    if sx == 0 and sy == 0 and sz == 0 and eps > 0.0:
                        g = g + (s2 + eps * eps) ** -1.5 - sv ** -3
                    w = np.where(keep, g * m[None, :], 0.0)
                    acc += np.einsum("tj,tjd->td", w, d)
        out[s:s + step] = acc
    return -G * out.T


def default_alpha(box):
    return 6.0 / box


def ewald_accel(pos, mass, box, G=1.0, eps=0.0, alpha=None, targets=None):
    """Periodic (Ewald) gravitational acceleration, shape (3, T)."""
    alpha = default_alpha(box) if alpha is None else alpha
    return (realspace_accel(pos, mass, box, alpha, G, eps, targets) +
            kspace_accel(pos, mass, box, alpha, G, targets))


def ewald_force(pos, mass, box, G=1.0, eps=0.0, alpha=None, targets=None):
    a = ewald_accel(pos, mass, box, G, eps, alpha, targets)
    if np.ndim(mass) == 0:
        return a * float(mass)
    m = np.asarray(mass, dtype=np.float64)
    return a * (m if targets is None else m[np.asarray(targets)])


def ewald_potential(pos, mass, box, G=1.0, alpha=None, targets=None):
    """Periodic potential with neutralising background (no softening), shape (T,).

    phi_i = -G sum_j m_j [ sum_n' erfc(alpha |r_n|)/|r_n|
                           + (4 pi/L^3) sum_{k!=0} exp(-k^2/4alpha^2)/k^2 cos(k.r)
                           - pi/(alpha^2 L^3) ] + G m_i 2 alpha/sqrt(pi)
    where the primed sum leaves out (j = i, n = 0); the last term removes the
    self-interaction that the k-space sum includes."""
    alpha = default_alpha(box) if alpha is None else alpha
    x = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)
    n = x.shape[0]
    m = _as_mass(mass, n)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    r_max = _REAL_SPAN / alpha
    n_img = max(0, int(math.ceil(r_max / box - 0.5)))
    shifts = np.arange(-n_img, n_img + 1) * box
    phi = np.zeros(len(targets))
    for a, i in enumerate(targets):
        d0 = x[i] - x
        d0 -= box * np.round(d0 / box)
        for sx in shifts:
            for sy in shifts:
                for sz in shifts:
                    d = d0 + np.array([sx, sy, sz])
                    s = np.sqrt(np.einsum("jd,jd->j", d, d))
                    keep = s < r_max
                    if sx == 0 and sy == 0 and sz == 0:
                        keep[i] = False
                    phi[a] += np.sum(np.where(keep, m * erfc(alpha * np.where(keep, s, 1.0))
                                              / np.where(keep, s, 1.0), 0.0))
    nk = int(math.ceil(math.sqrt(_KSPACE_EXPONENT) * alpha * box / math.pi))
    vecs = _half_space_vectors(nk)
    kf = 2.0 * np.pi / box
    k = kf * vecs
    k2 = np.einsum("kd,kd->k", k, k)
    coef = np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    S = np.exp(1j * (x @ k.T)).T @ m                       # (K,)
    e_t = np.exp(1j * (x[targets] @ k.T))                  # (T, K)
    # sum_j m_j cos(k.(x_i - x_j)) = Re(e^{ik.x_i} conj S); half space -> x2
    phi += (4.0 * np.pi / box ** 3) * 2.0 * np.real(e_t * np.conj(S)[None, :]) @ coef
    phi -= np.pi / (alpha * alpha * box ** 3) * np.sum(m)
    return -G * phi + G * m[targets] * 2.0 * alpha / _SQRT_PI
