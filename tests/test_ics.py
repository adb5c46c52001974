"""Sanity of the synthetic input recipes (parity unpinned: inputs are shared
by both sides, so these only check that each recipe does what it states)."""
import numpy as np

from paper_1510_07621_amd import ics


def test_uniform_in_box_and_seeded():
    a = ics.uniform(1000, 2.0, seed=4)
    b = ics.uniform(1000, 2.0, seed=4)
    assert a.shape == (3, 1000) and a.flags.c_contiguous
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() < 2.0


def test_zeldovich_rms_displacement():
    pos, q, psi = ics.zeldovich_lattice(16, 1.0, seed=2, return_parts=True)
    rms = np.sqrt(np.mean(np.sum(psi ** 2, axis=0)))
    assert abs(rms - 0.3 / 16) < 1e-12
    assert np.allclose(ics.wrap_positions(q + psi, 1.0), pos)
    assert abs(np.mean(psi)) < 1e-12          # k = 0 mode removed
    assert pos.min() >= 0 and pos.max() < 1.0


def test_plummer_mix_counts_and_truncation():
    n = 20000
    pos, lab, centres, a = ics.plummer_mix(n, 1.0, seed=3, n_spheres=50, return_labels=True)
    assert np.count_nonzero(lab >= 0) == 14000
    assert a.min() >= 0.002 and a.max() <= 0.02
    d = pos.T[lab >= 0] - centres[lab[lab >= 0]]
    d -= np.round(d)
    r = np.linalg.norm(d, axis=1)
    assert np.all(r <= 10 * a[lab[lab >= 0]] * (1 + 1e-9))
    # Plummer half-mass radius ~ 1.305 a (of the untruncated profile)
    ratio = np.median(r / a[lab[lab >= 0]])
    assert 1.15 < ratio < 1.35
    assert pos.min() >= 0 and pos.max() < 1.0
