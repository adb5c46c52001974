"""Relative force-error statistics used to state parity.

For each particle e_i = |F_i - F_i^ref| / |F_i^ref|. The RMS and the
maximum are taken over the particles whose reference force is at least 1e-6
times the median reference magnitude (symmetric configurations can have
|F^ref| ~ 0, where a relative error means nothing); the number left out is
reported. The global ratio sqrt(sum |dF|^2 / sum |F^ref|^2) is reported too.
"""
from __future__ import annotations

import numpy as np


def force_errors(F, Fref, floor=1e-6):
    F = np.asarray(F, dtype=np.float64)
    Fref = np.asarray(Fref, dtype=np.float64)
    dn = np.sqrt(np.sum((F - Fref) ** 2, axis=0))
    rn = np.sqrt(np.sum(Fref ** 2, axis=0))
    med = float(np.median(rn)) if rn.size else 0.0
    ok = rn >= floor * med if med > 0 else np.zeros_like(rn, dtype=bool)
    e = np.where(ok, dn / np.where(ok, rn, 1.0), 0.0)
    n_ok = int(np.count_nonzero(ok))
    return {
        "rms": float(np.sqrt(np.sum(e[ok] ** 2) / n_ok)) if n_ok else 0.0,
        "max": float(np.max(e[ok])) if n_ok else 0.0,
        "global": float(np.sqrt(np.sum(dn ** 2) / max(np.sum(rn ** 2), 1e-300))),
        "n": int(rn.size),
        "excluded": int(rn.size - n_ok),
    }
