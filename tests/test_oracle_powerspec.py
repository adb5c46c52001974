"""Pins of the oracle's power spectrum and sigma(R).

Closed forms and identities the estimator must satisfy: Parseval (the mode
sum of the spectrum is the grid variance of the density contrast; sigma at
R = 0 is the same number), a lattice on the nodes has no power, a node
density with one cosine mode puts exactly L^3 eps^2 / 2 into that mode's
shell (divided by W^2 when deconvolved), Poisson noise of uniform random
particles follows the CIC alias sum L^3/N prod_d (1 - 2/3 sin^2(pi n_d/N_g)),
and the guide's own test (Ch. 8 powerspec): sigma from the spectrum against
the rms of particle counts in cubes of the sphere's volume.
"""
import math

import numpy as np
import pytest

from oracle import powerspec
from oracle.pm import cic_deposit
from paper_1510_07621_amd import ics


def _all_bins(ng):
    return int(math.ceil(math.sqrt(3.0) * ng / 2)) + 1


def test_parseval_and_sigma_at_zero_radius():
    ng, box = 16, 2.0
    pos = ics.uniform(3000, box=box, seed=61)
    m = np.random.default_rng(62).uniform(0.5, 1.5, 3000)
    k, P, modes, s0 = powerspec.power_spectrum(pos, m, box, ng, _all_bins(ng),
                                               deconvolve=False, r_tophat=0.0)
    rho = cic_deposit(pos, m, box, ng)
    delta = rho / (m.sum() / box ** 3) - 1.0
    var = np.mean(delta ** 2)
    assert np.sum(modes * P) / box ** 3 == pytest.approx(var, rel=1e-12)
    assert s0 ** 2 == pytest.approx(var, rel=1e-12)
    assert modes.sum() == ng ** 3 - 1                  # every mode but k = 0, once
    # each shell's mean |k| lies inside the shell
    live = modes > 0
    nmean = k[live] * box / (2 * np.pi)
    b = np.nonzero(live)[0]
    assert np.all((nmean >= b + 0.5 - 1e-12) & (nmean < b + 1.5))


def test_lattice_on_nodes_has_no_power():
    ng = 16
    pos = ics.lattice(ng)
    k, P, modes, s = powerspec.power_spectrum(pos, 1.0, 1.0, ng, ng // 2, r_tophat=0.1)
    assert np.max(np.abs(P)) < 1e-28 and s < 1e-14


@pytest.mark.parametrize("n0", [(3, 0, 0), (1, 2, 2), (0, 5, 7)])
def test_single_cosine_mode(n0):
    """Unit particles on the nodes weighted 1 + eps cos(k0 . c): the deposit is
    exact, delta = eps cos(k0 . c), so the shell of |n0| holds L^3 eps^2 / 2."""
    ng, box, eps = 16, 1.5, 0.01
    c = ics.lattice(ng, box=box)
    n0 = np.array(n0, dtype=np.float64)
    w = 1.0 + eps * np.cos(2 * np.pi / box * (n0 @ c))
    nb = _all_bins(ng)
    b0 = int(np.floor(np.linalg.norm(n0) - 0.5))
    for deconv in (False, True):
        k, P, modes, _ = powerspec.power_spectrum(c, w, box, ng, nb, deconvolve=deconv)
        total = modes * P
        W = np.prod(np.sinc(n0 / ng) ** 2)
        expect = box ** 3 * eps ** 2 / 2 / (W ** 2 if deconv else 1.0)
        assert total[b0] == pytest.approx(expect, rel=1e-9)
        others = np.delete(total, b0)
        assert np.max(np.abs(others)) < 1e-12 * expect


def test_poisson_noise_follows_the_cic_alias_sum():
    ng, n = 32, 65536
    pos = ics.uniform(n, seed=63)
    nb = 12
    k, P, modes, _ = powerspec.power_spectrum(pos, 1.0 / n, 1.0, ng, nb, deconvolve=False)
    # expected raw power per shell: L^3/N times the shell mean of the alias sum
    C = powerspec.cic_shot_noise_factor(ng)
    nx, ny, nz, mult = powerspec._modes(ng)
    nabs = np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    b = np.floor(nabs - 0.5).astype(int)
    sel = (nabs > 0) & (b >= 0) & (b < nb)
    cm = np.bincount(b[sel], weights=(mult * C)[sel], minlength=nb) / modes
    ratio = np.sum((modes * P)[2:]) / np.sum((modes * cm)[2:] / n)
    assert abs(ratio - 1.0) < 0.03


def test_sigma_matches_counts_in_cubes():
    """The guide's powerspec test: sigma(R) from the spectrum against the rms
    of counts in cubes of the sphere's volume (side (4 pi / 3)^(1/3) R), for
    a lattice displaced by 1.5 spacings rms (so the lattice's own
    discreteness does not dominate the counts); sphere and cube windows
    differ, so the two agree to a few percent (1.5 % here)."""
    ng = 64
    pos = ics.zeldovich_lattice(ng, seed=64, rms_frac=1.5)
    side_cells = 8
    R = side_cells / ng / (4 * np.pi / 3) ** (1 / 3)
    _, _, _, sig = powerspec.power_spectrum(pos, 1.0, 1.0, ng, 4, deconvolve=True,
                                            r_tophat=R)
    counts = np.histogramdd(pos.T, bins=ng, range=[(0, 1)] * 3)[0]
    # counts in every cube of side_cells^3 cells (periodic, overlapping)
    c = counts
    for ax in range(3):
        c = sum(np.roll(c, -s, axis=ax) for s in range(side_cells))
    mean = side_cells ** 3 * pos.shape[1] / ng ** 3
    rms = np.std(c / mean - 1.0)
    assert abs(sig / rms - 1.0) < 0.05
