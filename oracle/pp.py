"""O-PP: the truncated short-range pair sum of P3M, by brute force.

Definition (guide Ch. 5: P3M short-range part cut off at r_c = P3M_cutoff *
r_s, Plummer softening of radius eps; split form from ``split``):

    r_ij = x_i - x_j - L * round((x_i - x_j) / L)          (minimum image)
    a_i  = -G * sum_{j != i, |r_ij| < r_c} m_j r_ij f(|r_ij|) / (|r_ij|^2 + eps^2)^(3/2)

Readings where the guide is silent: the cutoff is strict (r < r_c); the pair
set uses the minimum image, which needs r_c < L/2; f is evaluated at the
unsoftened distance; a pair at zero separation contributes nothing (its
r_ij is the zero vector).

Two neighbour searches give the identical pair set: an all-pairs scan
(``method="brute"``) and scipy's periodic k-d tree (``method="kdtree"``),
whose candidate list is then filtered with the same strict test.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .split import split_factor


def _as_mass(mass, n):
    if np.ndim(mass) == 0:
        return np.full(n, float(mass))
    return np.asarray(mass, dtype=np.float64)


def _pair_accel(xi, xj, mj, box, r_s, r_c, eps, G):
    """Accelerations on targets xi (T,3) from the listed partners.

    xj is (T, K, 3) and mj (T, K), padded entries carry mj = 0."""
    d = xi[:, None, :] - xj
    d -= box * np.round(d / box)
    r2 = np.einsum("tkd,tkd->tk", d, d)
    keep = (r2 < r_c * r_c) & (r2 > 0.0) & (mj != 0.0)
    r2k = np.where(keep, r2, 1.0)
    w = np.where(keep, mj * split_factor(np.sqrt(r2k), r_s) / (r2k + eps * eps) ** 1.5, 0.0)
    return -G * np.einsum("tk,tkd->td", w, d)


def pp_accel(pos, mass, box, r_s, r_c, eps, G=1.0, targets=None, method="auto",
             chunk=None):
    """Short-range P3M acceleration, shape (3, T) for the target indices.

    pos: (3, N) float64 in [0, box); mass: (N,) or scalar."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    if not (r_c < 0.5 * box):
        raise ValueError("minimum-image pair sum needs r_c < box/2")
    m = _as_mass(mass, n)
    x = np.ascontiguousarray(pos.T)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    out = np.zeros((len(targets), 3))
    if method == "auto":
        method = "brute" if n <= 2048 else "kdtree"
    if method == "brute":
        step = chunk or max(1, 2_000_000 // max(n, 1))
        for s in range(0, len(targets), step):
            t = targets[s:s + step]
            mj = np.broadcast_to(m, (len(t), n)).copy()
            mj[np.arange(len(t)), t] = 0.0       # j != i
            out[s:s + step] = _pair_accel(x[t], x[None, :, :], mj, box, r_s,
                                          r_c, eps, G)
        return np.ascontiguousarray(out.T)
    if method != "kdtree":
        raise ValueError(method)
    tree = cKDTree(x, boxsize=box)
    step = chunk or 4096
    for s in range(0, len(targets), step):
        t = targets[s:s + step]
        lists = tree.query_ball_point(x[t], r_c)
        lens = np.fromiter((len(lst) for lst in lists), dtype=np.int64, count=len(t))
        rows = np.repeat(np.arange(len(t)), lens)
        cols = (np.concatenate([np.asarray(lst, dtype=np.int64) for lst in lists])
                if lens.sum() else np.zeros(0, dtype=np.int64))
        d = x[t][rows] - x[cols]
        d -= box * np.round(d / box)
        r2 = np.einsum("kd,kd->k", d, d)
        keep = (r2 < r_c * r_c) & (r2 > 0.0) & (cols != t[rows])
        rows, cols, d, r2 = rows[keep], cols[keep], d[keep], r2[keep]
        w = m[cols] * split_factor(np.sqrt(r2), r_s) / (r2 + eps * eps) ** 1.5
        acc = np.zeros((len(t), 3))
        for dim in range(3):
            acc[:, dim] = np.bincount(rows, weights=w * d[:, dim], minlength=len(t))
        out[s:s + step] = -G * acc
    return np.ascontiguousarray(out.T)


def count_pairs(pos, box, r_c, targets=None):
    """Number of ordered pairs (i in targets, j != i) with minimum-image r < r_c."""
    pos = np.asarray(pos, dtype=np.float64)
    x = np.ascontiguousarray(pos.T)
    n = x.shape[0]
    targets = np.arange(n) if targets is None else np.asarray(targets)
    tree = cKDTree(x, boxsize=box)
    total = 0
    for s in range(0, len(targets), 8192):
        t = targets[s:s + 8192]
        lists = tree.query_ball_point(x[t], r_c)
        for i, lst in zip(t, lists):
            if not lst:
                continue
            j = np.asarray(lst)
            d = x[i] - x[j]
            d -= box * np.round(d / box)
            r2 = np.einsum("kd,kd->k", d, d)
            total += int(np.count_nonzero((r2 < r_c * r_c) & (j != i)))
    return total
