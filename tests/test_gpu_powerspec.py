"""GPU parity of the power spectrum (p3m_power_spectrum) against the oracle.

Same inputs, same estimator: shell-mean power per unit-width shell, the
shells' mean |k| and mode counts, and sigma(R). FP64 plans agree to 1e-10
(relative, per shell); FP32 plans (FP32 deposit and FFT) to 1e-3 on shells
holding at least 1e-6 of the peak power; mode counts exactly.
"""
import numpy as np
import pytest

from oracle import powerspec
from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _compare(got, ref, tol_p, tol_s):
    k, P, modes, sig = got
    rk, rP, rmodes, rsig = ref
    np.testing.assert_array_equal(modes, rmodes)
    live = rmodes > 0
    np.testing.assert_allclose(k[live], rk[live], rtol=1e-12)
    big = live & (rP >= 1e-6 * rP.max())
    assert np.max(np.abs(P[big] / rP[big] - 1.0)) <= tol_p
    assert abs(sig / rsig - 1.0) <= tol_s


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-3)])
@pytest.mark.parametrize("deconv", [2, 0])
def test_power_spectrum_parity_zeldovich64(precision, tol, deconv):
    w = ics.workload("zeldovich64_kdk")
    pos = w.positions()
    R = 8.0 / 64
    ref = powerspec.power_spectrum(pos, w.mass, 1.0, 64, 48, deconvolve=deconv != 0,
                                   r_tophat=R)
    with plan(64, w.n, precision, deconv_power=deconv) as P:
        k, p, m, s = P.power_spectrum(dev(pos), w.mass, nbins=48, r_tophat=R)
        got = (host(k), host(p), host(m), float(host(s)))
    _compare(got, ref, tol, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-3)])
def test_power_spectrum_parity_zeldovich128_bench_configuration(precision, tol):
    """The full-size call the bench times: 128^3 particles, 128^3 grid, the
    default 64 shells, sigma at 8 cells."""
    w = ics.workload("zeldovich128")
    pos = w.positions()
    R = 8.0 / 128
    ref = powerspec.power_spectrum(pos, w.mass, 1.0, 128, 64, r_tophat=R)
    with plan(128, w.n, precision) as P:
        k, p, m, s = P.power_spectrum(dev(pos), w.mass, r_tophat=R)
        got = (host(k), host(p), host(m), float(host(s)))
    assert got[1].shape == (64,)
    _compare(got, ref, tol, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-3)])
def test_power_spectrum_parity_clustered_masses_and_all_shells(precision, tol):
    """Plummer-clustered particles with per-particle masses on a 32^3 grid in
    a box of side 3, every shell out to the grid's corner, and R = 0 (the
    grid variance)."""
    n, ng, box = 20000, 32, 3.0
    pos = ics.plummer_mix(n, box=box, seed=71, n_spheres=20)
    m = np.random.default_rng(72).uniform(0.5, 1.5, n)
    nb = int(np.ceil(np.sqrt(3.0) * ng / 2)) + 1
    ref = powerspec.power_spectrum(pos, m, box, ng, nb, r_tophat=0.0)
    with plan(ng, n, precision, box=box) as P:
        k, p, mm, s = P.power_spectrum(dev(pos), dev(m), nbins=nb)
        got = (host(k), host(p), host(mm), float(host(s)))
    assert got[2].sum() == ng ** 3 - 1
    _compare(got, ref, tol, tol)


def test_power_spectrum_argument_errors():
    pos = dev(ics.uniform(100, seed=73))
    with plan(16, 100, "fp64") as P:
        for kw in (dict(nbins=0), dict(nbins=513), dict(r_tophat=-1.0),
                   dict(r_tophat=float("nan"))):
            with pytest.raises(ValueError):
                P.power_spectrum(pos, 0.01, **kw)
        with pytest.raises(ValueError):
            P.power_spectrum(pos[:, :0].contiguous(), 0.01)
        with pytest.raises(ValueError):
            P.power_spectrum(pos, 0.0)                  # no mass
