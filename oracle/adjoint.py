"""Adjoint (vector-Jacobian product) of the P3M force and of the leapfrog.

The guide's simulations advance particles with kicks and drifts driven by
the P3M force (CONCEPT User's Guide, Ch. 5: kick_algorithms, P3M; Ch. 6:
comoving positions and momenta). It gives no derivatives; what is written
here is the exact transpose of the forward definitions in ``pp``, ``pm`` and
``integrate``, so that for any cotangent lam (3, N) on the force,

    pos_bar_k = sum_i lam_i . dF_i / dx_k,      F_i = m_i (a_PP,i + a_PM,i).

Short range. With r = x_k - x_j (minimum image), rho^2 = r^2 + eps^2,
g(r) = f(r) / rho^3 and the pair Jacobian J = g I + (g'(r) / r) r r^T
(symmetric, even in r):

    pos_bar_k = -G m_k sum_{j: 0 < r < r_c} m_j J(r_kj) (lam_k - lam_j),
    g'(r) / r = f'(r) / (r rho^3) - 3 f / rho^5,
    f'(r) = -(r^2 / (2 sqrt(pi) r_s^3)) exp(-r^2 / (4 r_s^2)).

The cutoff makes F jump where a pair crosses r_c (f(r_c) != 0); the
derivative is the one away from those crossings.

Long range. a_PM(x) = -sum_c W(x - c) E(c), E = D phi, phi = P rho,
rho(c) = h^-3 sum_j m_j W(x_j - c), with P the Fourier-space Green's function
operator (real, even multiplier: P^T = P) and D the central difference
(D_d^T = -D_d). Then

    pos_bar_k = m_k sum_c grad W(x_k - c) [h^-3 psi(c) - lam_k . E(c)],
    psi = P S,  S = sum_d D_d Lam_d,  Lam_d(c) = sum_i m_i lam_{i,d} W(x_i - c).

The first term is the change of the density the particle deposits, the
second the change of its own interpolation weights. CIC weights are
piecewise linear, so this is the derivative away from node planes.

Leapfrog. One kick-drift-kick step (static background, ``integrate``):
p' = p + (dt/2) F(x), x1 = wrap(x + dt p' / m), p1 = p' + (dt/2) F(x1). Its
transpose, from (x1_bar, p1_bar) back to (x_bar, p_bar), in reverse order:

    x1_bar += VJP_F(x1, (dt/2) p1_bar);   p'_bar = p1_bar
    p'_bar += (dt / m) x1_bar;            x_bar = x1_bar      (wrap: slope 1)
    x_bar  += VJP_F(x, (dt/2) p'_bar);    p_bar = p'_bar

TEST INFRASTRUCTURE ONLY: the GPU path neither imports nor calls this.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .pm import cic_weights, fd_gradient, potential
from .split import SQRT_PI, split_factor
from . import integrate


def _as_mass(mass, n):
    if np.ndim(mass) == 0:
        return np.full(n, float(mass))
    return np.asarray(mass, dtype=np.float64)


def split_factor_derivative(r, r_s):
    """df/dr of the short-range share f(r) (float64)."""
    r = np.asarray(r, dtype=np.float64)
    return -(r * r / (2.0 * SQRT_PI * r_s ** 3)) * np.exp(-r * r / (4.0 * r_s * r_s))


def _pairs(pos, box, r_c, method="auto"):
    """All ordered pairs (i, j), i != j, at minimum-image distance 0 < r < r_c:
    an all-pairs scan (``brute``) or scipy's periodic k-d tree (``kdtree``)."""
    n = pos.shape[1]
    x = np.ascontiguousarray(pos.T)
    if method == "auto":
        method = "brute" if n <= 2048 else "kdtree"
    if method == "brute":
        i, j = np.nonzero(~np.eye(n, dtype=bool))
    else:
        tree = cKDTree(x, boxsize=box)
        pr = tree.query_pairs(r_c, output_type="ndarray")
        i = np.concatenate([pr[:, 0], pr[:, 1]])
        j = np.concatenate([pr[:, 1], pr[:, 0]])
    d = x[i] - x[j]
    d -= box * np.round(d / box)
    r2 = np.einsum("pd,pd->p", d, d)
    keep = (r2 < r_c * r_c) & (r2 > 0.0)
    return i[keep], j[keep], d[keep], r2[keep]


def _pairs_of(pos, targets, box, r_c):
    """Pairs (t, j) with t indexing ``targets``: every j at minimum-image
    distance 0 < r < r_c from particle targets[t] (periodic k-d tree)."""
    x = np.ascontiguousarray(pos.T)
    tg = np.asarray(targets)
    lists = cKDTree(x, boxsize=box).query_ball_point(x[tg], r_c)
    t = np.repeat(np.arange(tg.size), [len(l) for l in lists])
    j = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists]) if t.size else t
    d = x[tg[t]] - x[j]
    d -= box * np.round(d / box)
    r2 = np.einsum("pd,pd->p", d, d)
    keep = (r2 < r_c * r_c) & (r2 > 0.0)
    return t[keep], j[keep], d[keep], r2[keep]


def pp_vjp(pos, mass, box, r_s, r_c, eps, lam, G=1.0, method="auto", targets=None):
    """pos_bar (3, N) of the short-range force m_i a_PP,i for cotangent lam (3, N);
    with ``targets``, only those particles' columns (3, len(targets)), from
    their own pairs."""
    pos = np.asarray(pos, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = pos.shape[1]
    if not (r_c < 0.5 * box):
        raise ValueError("minimum-image pair sum needs r_c < box/2")
    m = _as_mass(mass, n)
    if targets is None:
        i, j, d, r2 = _pairs(pos, box, r_c, method)
        k, rows = i, n
    else:
        tg = np.asarray(targets)
        i, j, d, r2 = _pairs_of(pos, tg, box, r_c)
        k, rows = tg[i], tg.size
    r = np.sqrt(r2)
    rho2 = r2 + eps * eps
    f = split_factor(r, r_s)
    fp = split_factor_derivative(r, r_s)
    g = f / rho2 ** 1.5
    g_over_r = fp / (r * rho2 ** 1.5) - 3.0 * f / rho2 ** 2.5   # g'(r) / r
    dl = lam[:, k].T - lam[:, j].T                               # (P, 3)
    rdl = np.einsum("pd,pd->p", d, dl)
    contrib = g[:, None] * dl + (g_over_r * rdl)[:, None] * d    # J (lam_k - lam_j)
    contrib *= m[j][:, None]
    out = np.zeros((rows, 3))
    np.add.at(out, i, contrib)
    mk = m if targets is None else m[np.asarray(targets)]
    return -G * mk[None, :] * out.T


def cic_weight_gradients(pos, box, ng):
    """Yield (flat node index, weight, grad weight (3, N)) for the 8 CIC corners."""
    h = box / ng
    i0, frac = cic_weights(pos, box, ng)
    for a in (0, 1):
        ix = (i0[0] + a) % ng
        wx = frac[0] if a else 1.0 - frac[0]
        dx = (1.0 if a else -1.0) / h
        for b in (0, 1):
            iy = (i0[1] + b) % ng
            wy = frac[1] if b else 1.0 - frac[1]
            dy = (1.0 if b else -1.0) / h
            for c in (0, 1):
                iz = (i0[2] + c) % ng
                wz = frac[2] if c else 1.0 - frac[2]
                dz = (1.0 if c else -1.0) / h
                grad = np.stack([dx * wy * wz, wx * dy * wz, wx * wy * dz])
                yield (ix * ng + iy) * ng + iz, wx * wy * wz, grad


def pm_vjp(pos, mass, box, ng, r_s, lam, G=1.0, fd_order=4, deconv_power=2):
    """pos_bar (3, N) of the long-range force m_i a_PM,i for cotangent lam (3, N)."""
    from .pm import cic_deposit
    pos = np.asarray(pos, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = pos.shape[1]
    m = _as_mass(mass, n)
    h = box / ng
    # forward potential gradient on the nodes
    phi = potential(cic_deposit(pos, m, box, ng), box, r_s, G, deconv_power)
    E = fd_gradient(phi, box, fd_order).reshape(3, -1)
    # Lam_d(c) = sum_i m_i lam_{i,d} W(x_i - c)
    Lam = np.zeros((3, ng ** 3))
    for flat, w, _ in cic_weight_gradients(pos, box, ng):
        for d in range(3):
            Lam[d] += np.bincount(flat, weights=m * lam[d] * w, minlength=ng ** 3)
    # S = sum_d D_d Lam_d, psi = P S
    S = fd_gradient(Lam[0].reshape(ng, ng, ng), box, fd_order)[0]
    S = S + fd_gradient(Lam[1].reshape(ng, ng, ng), box, fd_order)[1]
    S = S + fd_gradient(Lam[2].reshape(ng, ng, ng), box, fd_order)[2]
    psi = potential(S, box, r_s, G, deconv_power).reshape(-1)
    out = np.zeros((3, n))
    for flat, _, grad in cic_weight_gradients(pos, box, ng):
        s = psi[flat] / h ** 3 - np.einsum("dn,dn->n", lam, E[:, flat])
        out += grad * s[None, :]
    return m[None, :] * out


def p3m_vjp(pos, mass, box, ng, lam, rs_cells=1.25, cutoff_rs=4.5, eps=0.0, G=1.0,
            fd_order=4, deconv_power=2):
    """pos_bar (3, N) of the P3M force F = m (a_PP + a_PM)."""
    h = box / ng
    r_s = rs_cells * h
    r_c = cutoff_rs * r_s
    return (pp_vjp(pos, mass, box, r_s, r_c, eps, lam, G) +
            pm_vjp(pos, mass, box, ng, r_s, lam, G, fd_order, deconv_power))


def leapfrog(pos, mom, mass, force_fn, dt, box, steps):
    """The forward trajectory: positions x_0..x_steps and the final momenta."""
    xs = [np.asarray(pos, dtype=np.float64)]
    p = np.asarray(mom, dtype=np.float64)
    F = None
    for _ in range(steps):
        x, p, F = integrate.kdk_step(xs[-1], p, mass, force_fn, dt, box, force=F)
        xs.append(x)
    return xs, p


def leapfrog_vjp(xs, mass, vjp_fn, dt, x_bar, p_bar):
    """Transpose of ``leapfrog`` given its positions xs; returns (x0_bar, p0_bar).

    ``vjp_fn(x, lam) -> pos_bar`` is the force VJP at positions x."""
    n = xs[0].shape[1]
    m = float(mass) if np.ndim(mass) == 0 else np.asarray(mass, dtype=np.float64)[None, :]
    xb = np.array(x_bar, dtype=np.float64)
    pb = np.array(p_bar, dtype=np.float64)
    assert xb.shape == (3, n) and pb.shape == (3, n)
    for t in range(len(xs) - 2, -1, -1):
        xb = xb + vjp_fn(xs[t + 1], 0.5 * dt * pb)     # second kick
        pb = pb + (dt / m) * xb                         # drift
        xb = xb + vjp_fn(xs[t], 0.5 * dt * pb)          # first kick
    return xb, pb
