"""Comoving kick/drift coefficients of the library (host code) against closed
forms of the Einstein-de Sitter and flat Lambda-CDM backgrounds and against
the oracle's independent quadrature (guide Ch. 5: H0, Omega_m, Omega_Lambda,
Delta t_factor; Ch. 6: comoving momenta)."""
import math
import os

import pytest

from oracle import cosmology as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(ROOT, "paper_1510_07621_amd", "libp3m.so")),
    reason="libp3m.so not built")


@pytest.fixture(scope="module")
def b():
    from paper_1510_07621_amd import binding
    return binding


def test_einstein_de_sitter_closed_forms(b):
    c = b.Cosmology(H0=0.7, Omega_m=1.0, Omega_L=0.0)
    for a in (1e-3, 0.02, 0.5, 1.0, 3.0):
        assert c.age(a) == pytest.approx(2.0 / (3.0 * 0.7) * a ** 1.5, rel=1e-12)
    for a0, a1 in ((0.01, 0.0125), (0.5, 1.0), (1e-3, 2e-3)):
        ck, cd = c.kick_drift(a0, a1)
        assert ck == pytest.approx(2.0 * (math.sqrt(a1) - math.sqrt(a0)) / 0.7, rel=1e-12)
        assert cd == pytest.approx(2.0 * (1 / math.sqrt(a0) - 1 / math.sqrt(a1)) / 0.7, rel=1e-12)


def test_flat_lcdm_age_closed_form(b):
    H0, Om, OL = 1.0, 0.3, 0.7
    c = b.Cosmology(H0, Om, OL)
    for a in (0.01, 0.1, 1.0):
        ref = 2.0 / (3.0 * H0 * math.sqrt(OL)) * math.asinh(math.sqrt(OL / Om) * a ** 1.5)
        assert c.age(a) == pytest.approx(ref, rel=1e-12)
        assert c.scale_factor(ref) == pytest.approx(a, rel=1e-12)


@pytest.mark.parametrize("Om,OL", [(0.3, 0.7), (0.3, 0.0), (1.2, 0.0), (0.25, 0.6)])
def test_coefficients_match_oracle_quadrature(b, Om, OL):
    c = b.Cosmology(0.9, Om, OL)
    for a0, a1 in ((0.02, 0.021), (0.1, 0.3), (0.5, 0.9)):
        ck, cd = c.kick_drift(a0, a1)
        rk, rd = oc.kick_drift(a0, a1, 0.9, Om, OL)
        assert ck == pytest.approx(rk, rel=1e-11)
        assert cd == pytest.approx(rd, rel=1e-11)
    assert c.age(0.7) == pytest.approx(oc.age(0.7, 0.9, Om, OL), rel=1e-11)


def test_kdk_step_covers_the_time_step(b):
    """Delta t = factor x age; the two kicks add up to the full-step kick."""
    c = b.Cosmology(1.0, 0.3, 0.7)
    a = 0.02
    a_next, k1, d, k2 = c.kdk_step(a, 0.01)
    assert c.age(a_next) == pytest.approx(1.01 * c.age(a), rel=1e-12)
    kf, df = c.kick_drift(a, a_next)
    assert k1 + k2 == pytest.approx(kf, rel=1e-12)
    assert d == pytest.approx(df, rel=1e-14)
    assert k1 > k2 > 0            # 1/a falls during the step


def test_cosmology_errors(b):
    import ctypes
    cs = b.P3MCosmology(1.0, 0.3, 0.7)
    out = ctypes.c_double()
    assert b._lib.p3m_cosmo_age(None, 1.0, ctypes.byref(out)) == -1
    assert b._lib.p3m_cosmo_age(ctypes.byref(cs), 0.0, ctypes.byref(out)) == -1
    assert b._lib.p3m_cosmo_kick_drift(ctypes.byref(cs), 0.5, 0.4, ctypes.byref(out),
                                      ctypes.byref(out)) == -1
    bad = b.P3MCosmology(-1.0, 0.3, 0.7)
    assert b._lib.p3m_cosmo_age(ctypes.byref(bad), 1.0, ctypes.byref(out)) == -1
    closed = b.P3MCosmology(1.0, 3.0, -2.5)   # recollapses before a = 2: H^2 < 0
    assert b._lib.p3m_cosmo_kick_drift(ctypes.byref(closed), 1.0, 3.0, ctypes.byref(out),
                                      ctypes.byref(out)) == -4
    with pytest.raises(ValueError):
        b.Cosmology(1.0, 0.3, 0.7).age(-1.0)


def test_kdk_step_einstein_de_sitter_closed_form(b):
    """Omega_m = 1: a(t) = (3 H0 t / 2)^(2/3), so a step of a fraction f of
    the age ends at a (1 + f)^(2/3) and its middle in time is at
    a (1 + f/2)^(2/3); the kicks and the drift are the closed-form
    integrals between them."""
    H0, a, f = 0.7, 0.05, 0.02
    c = b.Cosmology(H0, 1.0, 0.0)
    a1, k1, d, k2 = c.kdk_step(a, f)
    ah = a * (1 + 0.5 * f) ** (2.0 / 3.0)
    assert a1 == pytest.approx(a * (1 + f) ** (2.0 / 3.0), rel=1e-12)
    assert k1 == pytest.approx(2.0 * (math.sqrt(ah) - math.sqrt(a)) / H0, rel=1e-11)
    assert k2 == pytest.approx(2.0 * (math.sqrt(a1) - math.sqrt(ah)) / H0, rel=1e-11)
    assert d == pytest.approx(2.0 * (1 / math.sqrt(a) - 1 / math.sqrt(a1)) / H0, rel=1e-11)


def test_kdk_step_matches_oracle_composition(b):
    """Flat Lambda-CDM: the library's step against the same composition of
    the oracle's quadrature and root finding."""
    H0, Om, OL, a, f = 1.0, 0.3, 0.7, 0.1, 0.03
    a1, k1, d, k2 = b.Cosmology(H0, Om, OL).kdk_step(a, f)
    t0 = oc.age(a, H0, Om, OL)
    ah = oc.scale_factor(t0 + 0.5 * f * t0, H0, Om, OL)
    ae = oc.scale_factor(t0 + f * t0, H0, Om, OL)
    assert a1 == pytest.approx(ae, rel=1e-11)
    assert k1 == pytest.approx(oc.kick_drift(a, ah, H0, Om, OL)[0], rel=1e-10)
    assert k2 == pytest.approx(oc.kick_drift(ah, ae, H0, Om, OL)[0], rel=1e-10)
    assert d == pytest.approx(oc.kick_drift(a, ae, H0, Om, OL)[1], rel=1e-10)


def test_kdk_step_errors(b):
    import ctypes
    cs = b.P3MCosmology(1.0, 0.3, 0.7)
    o = [ctypes.c_double() for _ in range(4)]
    ref = [ctypes.byref(x) for x in o]
    L = b._lib
    assert L.p3m_cosmo_kdk_step(None, 0.1, 0.01, *ref) == -1
    assert L.p3m_cosmo_kdk_step(ctypes.byref(cs), 0.0, 0.01, *ref) == -1
    assert L.p3m_cosmo_kdk_step(ctypes.byref(cs), 0.1, 0.0, *ref) == -1
    assert L.p3m_cosmo_kdk_step(ctypes.byref(cs), 0.1, float("nan"), *ref) == -1
    assert L.p3m_cosmo_kdk_step(ctypes.byref(cs), 0.1, 0.01, None, ref[1], ref[2], ref[3]) == -1
    with pytest.raises(ValueError):
        b.Cosmology(1.0, 0.3, 0.7).kdk_step(0.1, -0.5)
