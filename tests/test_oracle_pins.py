"""Pins of the CPU reference against facts that do not come from itself.

Each test ties one oracle function to something the guide states, a closed
form, a published constant, a symmetry, or an independent computation
(e.g. the particle-mesh long range against the Fourier half of a direct Ewald
sum). They run on the CPU in a few seconds each.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import ewald, integrate as integ, metrics, p3m, pm, pp, split
from paper_1510_07621_amd import ics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- split factor

def test_split_cutoff_statement_of_the_guide():
    """Guide Ch. 5, P3M_cutoff: a cutoff >= 4.8 split scales drops < 1 % of the force.

    The reading (Gaussian split, u = r / 2 r_s) must make 4.8 the threshold:
    below 1 % at 4.8, above it a little earlier."""
    (cut, bound, rel), = _golden("split_cutoff_statement.txt")
    cut, bound = float(cut), float(bound)
    assert rel == "below"
    assert split.split_factor(cut, 1.0) < bound
    assert split.split_factor(cut - 0.05, 1.0) > bound
    # monotone decreasing from 1
    r = np.linspace(0.0, 8.0, 400)
    f = split.split_factor(r, 1.0)
    assert f[0] == 1.0 and np.all(np.diff(f) < 0)


def test_split_is_enclosed_mass_of_the_gaussian_cloud():
    """1 - f(r) is the mass fraction inside r of the Gaussian cloud whose
    potential has the Fourier kernel exp(-k^2 r_s^2)/k^2, i.e. a Gaussian of
    variance 2 r_s^2 per axis (checked by quadrature of the density)."""
    r_s = 0.7
    sig2 = 2.0 * r_s * r_s
    dens = lambda s: 4 * np.pi * s * s * np.exp(-s * s / (2 * sig2)) / (2 * np.pi * sig2) ** 1.5
    for r in (0.1, 0.5, 1.0, 2.0, 3.15):
        enclosed, _ = integrate.quad(dens, 0.0, r, epsabs=1e-14, epsrel=1e-13)
        assert abs((1.0 - split.split_factor(r, r_s)) - enclosed) < 1e-12


# ---------------------------------------------------------------- Ewald truth

def test_ewald_two_body_small_separation():
    """Closed form |a| = G m / d^2 (1 - (4 pi / 3)(d/L)^3) + O((d/L)^5):
    cubic symmetry removes the images' tidal term, the background pulls out."""
    for d, tol in ((0.01, 1e-8), (0.05, 2e-5)):
        pos = np.array([[0.3, 0.3 + d], [0.4, 0.4], [0.5, 0.5]])
        a = ewald.ewald_accel(pos, 1.0, 1.0)
        ref = 1.0 / d ** 2 * (1.0 - 4.0 * math.pi / 3.0 * d ** 3)
        assert a[0, 0] > 0 and a[0, 1] < 0          # attraction
        assert abs(a[0, 0] - ref) / ref < tol
        assert np.max(np.abs(a[1:])) < 1e-12 * ref


def test_ewald_independent_of_alpha():
    rng = np.random.default_rng(11)
    pos = rng.random((3, 40))
    m = rng.random(40)
    ref = ewald.ewald_accel(pos, m, 1.0, alpha=5.0, eps=1e-3)
    for alpha in (3.0, 7.5):
        a = ewald.ewald_accel(pos, m, 1.0, alpha=alpha, eps=1e-3)
        assert np.max(np.abs(a - ref)) < 1e-12 * np.max(np.abs(ref))


def test_ewald_madelung_constant():
    (val, tol), = _golden("madelung_simple_cubic.txt")
    for alpha in (4.0, 6.0):
        phi = ewald.ewald_potential(np.array([[0.2], [0.3], [0.4]]), 1.0, 1.0, alpha=alpha)
        assert abs(phi[0] - float(val)) < float(tol)


def test_ewald_symmetric_configurations_have_zero_force():
    lat = ics.lattice(4, offset=0.3)
    a = ewald.ewald_accel(lat, 1.0, 1.0)
    assert np.max(np.abs(a)) < 1e-11
    for second in ([0.6, 0.2, 0.3], [0.6, 0.7, 0.8]):     # (L/2,0,0), (L/2,L/2,L/2)
        pos = np.array([[0.1, second[0]], [0.2, second[1]], [0.3, second[2]]])
        assert np.max(np.abs(ewald.ewald_accel(pos, 1.0, 1.0))) < 1e-12


def test_ewald_plummer_softening_two_body():
    """Close pair with softening: a = G m d / (d^2 + eps^2)^(3/2) minus the
    background term (images negligible at this separation)."""
    d, eps = 0.004, 0.003
    pos = np.array([[0.5, 0.5 + d], [0.5, 0.5], [0.5, 0.5]])
    a = ewald.ewald_accel(pos, 1.0, 1.0, eps=eps)
    ref = d / (d * d + eps * eps) ** 1.5 - 4.0 * math.pi / 3.0 * d
    assert abs(a[0, 0] - ref) / ref < 1e-9


# ---------------------------------------------------------------- short range

def test_pp_brute_equals_kdtree():
    pos = ics.uniform(1500, seed=5)
    m = np.random.default_rng(6).random(1500)
    args = (1.0, 0.03, 0.15, 2e-3)
    a1 = pp.pp_accel(pos, m, *args, method="brute")
    a2 = pp.pp_accel(pos, m, *args, method="kdtree")
    assert np.max(np.abs(a1 - a2)) <= 1e-13 * np.max(np.abs(a1))


def test_pp_equals_ewald_real_space_when_cutoff_is_wide():
    """With eps = 0 and a cutoff where f ~ 1e-17, the P3M short range is the
    real-space half of the Ewald sum at alpha = 1 / (2 r_s)."""
    pos = ics.uniform(1200, seed=8)
    r_s = 0.02
    a = pp.pp_accel(pos, 1.0, 1.0, r_s, 12 * r_s, 0.0)
    ref = ewald.realspace_accel(pos, 1.0, 1.0, alpha=1.0 / (2 * r_s))
    err = metrics.force_errors(a, ref)
    assert err["rms"] < 1e-13 and err["max"] < 1e-11


def test_pp_newton_third_law_and_lattice():
    pos = ics.uniform(1000, seed=9)
    m = np.random.default_rng(10).random(1000)
    a = pp.pp_accel(pos, m, 1.0, 0.04, 0.18, 1e-3)
    tot = np.sum(a * m, axis=1)
    assert np.max(np.abs(tot)) < 1e-12 * np.sum(np.abs(a * m))
    lat = ics.lattice(8, offset=0.25)
    assert np.max(np.abs(pp.pp_accel(lat, 1.0, 1.0, 0.1, 0.45, 0.0))) < 1e-10


def test_pp_cutoff_is_strict_and_minimum_image():
    r_s, r_c = 0.05, 0.2
    # partner across the face at minimum-image distance 0.1: inside
    pos = np.array([[0.02, 0.92], [0.5, 0.5], [0.5, 0.5]])
    a = pp.pp_accel(pos, 1.0, 1.0, r_s, r_c, 0.0)
    assert a[0, 0] < 0 and a[0, 1] > 0      # pulled towards -x / +x across the face
    # outside the cutoff: nothing
    pos = np.array([[0.1, 0.35], [0.5, 0.5], [0.5, 0.5]])
    assert np.all(pp.pp_accel(pos, 1.0, 1.0, r_s, r_c, 0.0) == 0.0)
    assert pp.count_pairs(ics.uniform(500, seed=3), 1.0, 0.1) > 0


# ---------------------------------------------------------------- mesh part

def test_cic_deposit_cases():
    ng, box = 8, 1.0
    h = box / ng
    # on a node: all mass on that node
    rho = pm.cic_deposit(np.array([[3 * h], [5 * h], [7 * h]]), 2.0, box, ng)
    assert rho[3, 5, 7] * h ** 3 == pytest.approx(2.0, abs=1e-14)
    assert np.count_nonzero(rho) == 1
    # at a cell centre: eight equal shares, wrapping through the top face
    rho = pm.cic_deposit(np.array([[7.5 * h], [0.5 * h], [2.5 * h]]), 1.0, box, ng)
    for ix in (7, 0):
        for iy in (0, 1):
            for iz in (2, 3):
                assert rho[ix, iy, iz] * h ** 3 == pytest.approx(0.125, abs=1e-15)
    # linear split along one axis
    rho = pm.cic_deposit(np.array([[1.25 * h], [0.0], [0.0]]), 1.0, box, ng)
    assert rho[1, 0, 0] * h ** 3 == pytest.approx(0.75)
    assert rho[2, 0, 0] * h ** 3 == pytest.approx(0.25)
    # mass conservation
    pos = ics.uniform(3000, seed=4)
    m = np.random.default_rng(1).random(3000)
    assert np.sum(pm.cic_deposit(pos, m, box, 16)) * (box / 16) ** 3 == pytest.approx(m.sum(), rel=1e-13)


def test_cic_interp_reproduces_constant_and_linear_fields():
    ng, box = 16, 2.0
    h = box / ng
    idx = np.arange(ng) * h
    X, Y, Z = np.meshgrid(idx, idx, idx, indexing="ij")
    fields = np.stack([np.full_like(X, 3.0), X, 2 * Y - Z])
    rng = np.random.default_rng(2)
    pos = rng.uniform(0.1, box - h - 0.1, (3, 200))     # away from the wrap
    out = pm.cic_interp(fields, pos, box)
    assert np.allclose(out[0], 3.0, atol=1e-14)
    assert np.allclose(out[1], pos[0], atol=1e-13)
    assert np.allclose(out[2], 2 * pos[1] - pos[2], atol=1e-13)


@pytest.mark.parametrize("order,coef", [(2, 1.0 / 6.0), (4, 1.0 / 30.0)])
def test_fd_gradient_truncation_error(order, coef):
    """Central differences of sin(kx): relative error ~ coef (kh)^order with
    coef = 1/6 (2-point) and 1/30 (4-point), the textbook leading terms."""
    ng, box = 64, 1.0
    h = box / ng
    n = 3
    k = 2 * np.pi * n / box
    x = np.arange(ng) * h
    phi = np.broadcast_to(np.sin(k * x)[None, None, :], (ng, ng, ng)).copy()
    g = pm.fd_gradient(phi, box, order)
    exact = k * np.cos(k * x)
    i = np.argmax(np.abs(exact))
    rel = (exact[i] - g[2, 0, 0, i]) / exact[i]
    lead = coef * (k * h) ** order
    assert 0.97 * lead < rel < 1.0 * lead
    assert np.max(np.abs(g[0])) < 1e-10 and np.max(np.abs(g[1])) < 1e-10


def test_pm_converges_to_ewald_fourier_part():
    """At fixed physical r_s, refining the mesh drives PM to the Fourier
    half of the Ewald sum with alpha = 1/(2 r_s)."""
    pos = ics.uniform(2048, seed=21)
    m = 1.0 / 2048
    r_s = 1.25 / 16
    tg = np.arange(0, 2048, 4)
    ref = ewald.kspace_accel(pos, m, 1.0, alpha=1.0 / (2 * r_s), targets=tg)
    errs = [metrics.force_errors(pm.pm_accel(pos, m, 1.0, ng, r_s, targets=tg), ref)["global"]
            for ng in (16, 32, 64)]
    assert errs[0] < 0.05 and errs[1] < 0.4 * errs[0] and errs[2] < 0.5 * errs[1]
    # the deconvolution and the 4-point gradient each lower the error
    no_dec = metrics.force_errors(pm.pm_accel(pos, m, 1.0, 32, r_s, deconv_power=0, targets=tg), ref)["global"]
    fd2 = metrics.force_errors(pm.pm_accel(pos, m, 1.0, 32, r_s, fd_order=2, targets=tg), ref)["global"]
    assert no_dec > 2 * errs[1] and fd2 > 2 * errs[1]


def test_pm_momentum_conservation_and_self_force():
    pos = ics.uniform(800, seed=12)
    m = np.random.default_rng(3).random(800)
    a = pm.pm_accel(pos, m, 1.0, 16, 1.25 / 16)
    tot = np.sum(a * m, axis=1)
    assert np.max(np.abs(tot)) < 1e-12 * np.sum(np.abs(a * m))
    for p in ([0.13, 0.77, 0.5], [0.031, 0.0, 0.999]):
        one = np.array(p, dtype=np.float64)[:, None]
        assert np.max(np.abs(pm.pm_accel(one, 1.0, 1.0, 16, 1.25 / 16))) < 1e-12


# ---------------------------------------------------------------- P3M

def test_p3m_approximates_ewald_truth():
    """The P3M method error against direct Ewald at the guide-style settings
    (split 1.25 cells, cutoff 4.5 r_s) is of order 1e-2 relative; widening the
    cutoff and refining the mesh at fixed r_s lowers it by more than 10x."""
    n = 2048
    pos = ics.uniform(n, seed=31)
    m = 1.0 / n
    eps = 0.03 / n ** (1 / 3)
    tg = np.arange(0, n, 4)
    ref = ewald.ewald_accel(pos, m, 1.0, eps=eps, targets=tg)
    base = metrics.force_errors(p3m.p3m_accel(pos, m, 1.0, 16, 1.25, 4.5, eps, targets=tg), ref)
    assert 1e-3 < base["rms"] < 3e-2
    # same physical r_s (1.25/16 = 5/64), 6 r_s cutoff, 4x finer mesh
    fine = metrics.force_errors(p3m.p3m_accel(pos, m, 1.0, 64, 5.0, 6.0, eps, targets=tg), ref)
    assert fine["rms"] < base["rms"] / 10


def test_p3m_lattice_and_plane_symmetry():
    lat = ics.lattice(8)
    a = p3m.p3m_accel(lat, 1.0 / 512, 1.0, 16, 1.25, 4.5, 1e-3)
    assert np.max(np.abs(a)) < 1e-10
    # density varying only along x (the guide's kick test design): no y, z force
    planes = ics.lattice(8)
    planes[0] = (planes[0] + 0.02 * np.sin(2 * np.pi * planes[0])) % 1.0
    a = p3m.p3m_accel(planes, 1.0 / 512, 1.0, 16, 1.25, 4.5, 1e-3)
    assert np.max(np.abs(a[1:])) < 1e-10 * np.max(np.abs(a[0]))
    assert np.max(np.abs(a[0])) > 1e-3


# ---------------------------------------------------------------- kick / drift

def test_drift_crossing_faces_closed_form():
    """Equal velocities on a lattice: every particle moves rigidly and
    crosses the box faces; after n steps x = wrap(x0 + n c v) to a few ulp."""
    pos = ics.lattice(4, offset=0.1)
    v = np.array([0.37, -0.81, 1.3])[:, None]
    m = 0.5
    mom = np.broadcast_to(v * m, pos.shape).copy()
    x = pos.copy()
    c = 0.173
    for _ in range(20):
        x = integ.drift(x, mom, m, c, 1.0)
    exact = integ.wrap(pos + 20 * c * v, 1.0)
    dist = np.abs(x - exact)
    dist = np.minimum(dist, 1.0 - dist)
    assert np.max(dist) < 1e-13
    assert np.all((x >= 0) & (x < 1.0))


def test_wrap_edges_and_kick():
    y = np.array([-1e-20, 1.0, 2.5, -0.25, 0.999999])
    w = integ.wrap(y, 1.0)
    assert list(w) == [0.0, 0.0, 0.5, 0.75, 0.999999]
    p = np.array([[1.0, 2.0]])
    f = np.array([[0.5, -4.0]], dtype=np.float32)
    assert np.all(integ.kick(p, f, 0.25) == np.array([[1.125, 1.0]]))


# ---------------------------------------------------------------- pair count

# Simple cubic lattice: the shells at squared distance 1, 2, 3, 4, 5 (in
# units of the spacing) hold 6, 12, 8, 6, 24 points, so the coordination
# number within a strict cutoff k * spacing is the sum over shells below k^2.
_SC_SHELLS = [(1, 6), (2, 12), (3, 8), (4, 6), (5, 24)]


@pytest.mark.parametrize("k,coord", [(1.5, 18), (1.8, 26), (2.1, 32), (2.3, 56)])
def test_count_pairs_simple_cubic_coordination(k, coord):
    """Ordered pairs on a periodic simple cubic lattice = N x coordination
    number (each neighbour seen from both sides, the point itself excluded)."""
    assert sum(c for d2, c in _SC_SHELLS if d2 < k * k) == coord
    n_side = 8
    lat = ics.lattice(n_side, offset=0.5)
    r_c = k / n_side
    assert pp.count_pairs(lat, 1.0, r_c) == n_side ** 3 * coord
    # a subset of targets counts its own rows only
    t = np.arange(0, n_side ** 3, 7)
    assert pp.count_pairs(lat, 1.0, r_c, targets=t) == t.size * coord


def test_count_pairs_brute_force_random():
    """Against an all-pairs count written out here on a small random set with
    two exact duplicates (separation 0 counts as a pair: j != i, r < r_c)."""
    rng = np.random.default_rng(41)
    pos = rng.random((3, 300)) * 1.3
    pos[:, 7] = pos[:, 3]
    pos[:, 250] = pos[:, 3]
    box, r_c = 1.3, 0.21
    n = pos.shape[1]
    count = 0
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d2 = 0.0
            for a in range(3):
                d = pos[a, i] - pos[a, j]
                d -= box * math.floor(d / box + 0.5)
                d2 += d * d
            count += d2 < r_c * r_c
    assert pp.count_pairs(pos, box, r_c) == count


# ---------------------------------------------------------------- error metric

def test_force_errors_hand_computed():
    """Four particles: relative errors 0.1, 0.05 and 0.2, and one particle
    whose reference force is below 1e-6 x the median (excluded from RMS and
    max, kept in the global ratio)."""
    ref = np.array([[1.0, 0.0, 0.0, 1e-9],
                    [0.0, 2.0, 0.0, 0.0],
                    [0.0, 0.0, 3.0, 0.0]])
    F = np.array([[1.1, 0.0, 0.0, 5.0],
                  [0.0, 2.0, 0.6, 0.0],
                  [0.0, 0.1, 3.0, 0.0]])
    e = metrics.force_errors(F, ref)
    assert e["n"] == 4 and e["excluded"] == 1
    assert e["max"] == pytest.approx(0.2, rel=1e-14)
    assert e["rms"] == pytest.approx(math.sqrt((0.01 + 0.0025 + 0.04) / 3.0), rel=1e-14)
    num = 0.01 + 0.01 + 0.36 + (5.0 - 1e-9) ** 2
    assert e["global"] == pytest.approx(math.sqrt(num / (1.0 + 4.0 + 9.0 + 1e-18)), rel=1e-14)
    # all references zero: nothing to compare, nothing reported as an error
    z = metrics.force_errors(F, np.zeros_like(ref))
    assert z["rms"] == 0.0 and z["max"] == 0.0 and z["excluded"] == 4


# ---------------------------------------------------------------- background

def test_oracle_cosmology_einstein_de_sitter():
    """Omega_m = 1: t = 2 a^(3/2) / (3 H0); int da / (a^2 H) = 2 (sqrt a1 -
    sqrt a0) / H0; int da / (a^3 H) = 2 (a0^-1/2 - a1^-1/2) / H0."""
    from oracle import cosmology as oc
    H0 = 0.7
    for a in (1e-3, 0.02, 0.5, 1.0, 3.0):
        t = 2.0 / (3.0 * H0) * a ** 1.5
        assert oc.age(a, H0, 1.0, 0.0) == pytest.approx(t, rel=1e-12)
        assert oc.scale_factor(t, H0, 1.0, 0.0) == pytest.approx(a, rel=1e-12)
    for a0, a1 in ((0.01, 0.0125), (0.5, 1.0), (1e-3, 2e-3)):
        ck, cd = oc.kick_drift(a0, a1, H0, 1.0, 0.0)
        assert ck == pytest.approx(2.0 * (math.sqrt(a1) - math.sqrt(a0)) / H0, rel=1e-12)
        assert cd == pytest.approx(2.0 * (1 / math.sqrt(a0) - 1 / math.sqrt(a1)) / H0, rel=1e-12)


def test_oracle_cosmology_flat_lcdm_and_empty_and_lambda_only():
    """Flat Lambda-CDM age: t = 2 asinh(sqrt(OL/Om) a^(3/2)) / (3 H0 sqrt OL).
    Empty (Milne, all curvature): H = H0 / a, t = a / H0, int dt/a =
    ln(a1/a0) / H0, int dt/a^2 = (1/a0 - 1/a1) / H0. Lambda only: H = H0,
    int dt/a = (1/a0 - 1/a1) / H0, int dt/a^2 = (a0^-2 - a1^-2) / (2 H0)."""
    from oracle import cosmology as oc
    H0, Om, OL = 1.3, 0.3, 0.7
    for a in (0.01, 0.1, 1.0):
        ref = 2.0 / (3.0 * H0 * math.sqrt(OL)) * math.asinh(math.sqrt(OL / Om) * a ** 1.5)
        assert oc.age(a, H0, Om, OL) == pytest.approx(ref, rel=1e-12)
        assert oc.scale_factor(ref, H0, Om, OL) == pytest.approx(a, rel=1e-12)
    for a0, a1 in ((0.02, 0.03), (0.5, 2.0)):
        assert oc.age(a1, H0, 0.0, 0.0) == pytest.approx(a1 / H0, rel=1e-12)
        ck, cd = oc.kick_drift(a0, a1, H0, 0.0, 0.0)
        assert ck == pytest.approx(math.log(a1 / a0) / H0, rel=1e-12)
        assert cd == pytest.approx((1 / a0 - 1 / a1) / H0, rel=1e-12)
        ck, cd = oc.kick_drift(a0, a1, H0, 0.0, 1.0)
        assert ck == pytest.approx((1 / a0 - 1 / a1) / H0, rel=1e-12)
        assert cd == pytest.approx((a0 ** -2 - a1 ** -2) / (2 * H0), rel=1e-12)
