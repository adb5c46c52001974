"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Element-by-element on the same seeded inputs. Tolerances (per-particle
relative force error, RMS over particles): FP64 path 1e-6 (checked tighter
where the arithmetic allows), FP32 path 1e-3; the short-range sum alone is
an exact sum reached faster, so it is held to 1e-12 (FP64) and 1e-5 (FP32).
Integer results (pair counts) are compared exactly; kick and drift bit for
bit.
"""
import numpy as np
import pytest
import torch

from oracle import ewald, integrate, metrics
from oracle import p3m as o_p3m
from oracle import pm as o_pm
from oracle import pp as o_pp
from paper_1510_07621_amd import ics

from _gpu import dev, host, oracle_parts, plan, require_gpu, sample_targets, workload_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _err(F, ref):
    return metrics.force_errors(F, ref)


# --------------------------------------------------------------- kick / drift

@pytest.mark.parametrize("n", [1, 1000, 65537])
def test_kick_bitwise(n):
    from paper_1510_07621_amd import binding
    rng = np.random.default_rng(n)
    p = rng.normal(size=(3, n))
    for fdt in (np.float64, np.float32):
        F = rng.normal(size=(3, n)).astype(fdt)
        pd = dev(p)
        binding.kick(pd, dev(F, torch.float64 if fdt == np.float64 else torch.float32), 0.37)
        assert np.array_equal(host(pd), integrate.kick(p, F, 0.37))


@pytest.mark.parametrize("use_mass_array", [False, True])
def test_kick_drift_fused_bitwise(use_mass_array):
    """The fused first half of a KDK step equals the oracle's kick followed by
    its drift bit for bit, for both force precisions, wrapping included."""
    from paper_1510_07621_amd import binding
    n = 4099                                    # not a multiple of the block
    rng = np.random.default_rng(9)
    x = ics.uniform(n, 1.0, seed=9)
    p = rng.normal(size=(3, n)) * 2.0
    m = rng.uniform(0.5, 2.0, n) if use_mass_array else 0.75
    for fdt in (np.float64, np.float32):
        F = rng.normal(size=(3, n)).astype(fdt)
        xd, pd = dev(x), dev(p)
        binding.kick_drift(xd, pd, dev(F, torch.float64 if fdt == np.float64 else torch.float32),
                           dev(m) if use_mass_array else m, 0.37, 0.61, 1.0)
        p1 = integrate.kick(p, F, 0.37)
        assert np.array_equal(host(pd), p1)
        assert np.array_equal(host(xd), integrate.drift(x, p1, m, 0.61, 1.0))
    with pytest.raises(ValueError):
        binding.kick_drift(dev(x), dev(p), dev(F[:, :10]), m, 0.1, 0.1, 1.0)


@pytest.mark.parametrize("use_mass_array", [False, True])
def test_drift_bitwise_and_wraps(use_mass_array):
    from paper_1510_07621_amd import binding
    n = 5000
    rng = np.random.default_rng(3)
    x = ics.uniform(n, 1.0, seed=3)
    p = rng.normal(size=(3, n)) * 2.0
    m = rng.uniform(0.5, 2.0, n) if use_mass_array else 0.75
    xd = dev(x)
    binding.drift(xd, dev(p), dev(m) if use_mass_array else m, 0.61, 1.0)
    got = host(xd)
    assert np.array_equal(got, integrate.drift(x, p, m, 0.61, 1.0))
    assert got.min() >= 0.0 and got.max() < 1.0


def test_drift_test_of_the_guide_crossing_faces():
    """Equal velocities on a lattice (no net force): 20 drifts through the
    faces equal the oracle bit for bit and the closed form to ~ulp."""
    from paper_1510_07621_amd import binding
    pos = ics.lattice(8, offset=0.1)
    v = np.array([0.37, -0.81, 1.3])[:, None]
    m = 0.5
    mom = np.broadcast_to(v * m, pos.shape).copy()
    xd, pd = dev(pos), dev(mom)
    x = pos.copy()
    for _ in range(20):
        binding.drift(xd, pd, m, 0.173, 1.0)
        x = integrate.drift(x, mom, m, 0.173, 1.0)
    got = host(xd)
    assert np.array_equal(got, x)
    exact = integrate.wrap(pos + 20 * 0.173 * v, 1.0)
    d = np.abs(got - exact)
    assert np.max(np.minimum(d, 1.0 - d)) < 1e-13


def test_comoving_kdk_steps_against_the_oracle():
    """Comoving leapfrog (guide Ch. 5: H0, Omega_m, Omega_Lambda, a_begin,
    Delta t_factor; Ch. 6: comoving positions and canonical momenta): three
    kick-drift-kick steps, each a fraction 0.05 of the age, from a = 0.02 in
    flat Lambda-CDM. The GPU takes the library's step coefficients and its
    FP64 P3M force; the oracle takes the same composition of its own
    quadrature (oracle.cosmology), its own P3M force and its own kick and
    drift. Positions agree to the force parity (1e-10 of a cell), momenta to
    1e-9 relative."""
    from oracle import cosmology as oc
    from paper_1510_07621_amd import binding
    H0, Om, OL, a0, f = 1.0, 0.3, 0.7, 0.02, 0.05
    grid, n = 16, 3000
    pos = ics.uniform(n, seed=77)
    m = 1.0 / n
    eps = 0.03 / 16
    cos = binding.Cosmology(H0, Om, OL)
    # GPU
    x = dev(pos)
    p = torch.zeros_like(x)
    with plan(grid, n, "fp64", softening=eps) as P:
        F = P.force(x, m)
        a = a0
        for _ in range(3):
            a1, k1, d, k2 = cos.kdk_step(a, f)
            binding.kick_drift(x, p, F, m, k1, d, 1.0)
            P.force(x, m, out=F)
            binding.kick(p, F, k2)
            a = a1
        xg, pg = host(x), host(p)
    # oracle
    xo, po = pos.copy(), np.zeros_like(pos)
    Fo = o_p3m.p3m_force(xo, m, 1.0, grid, 1.25, 4.5, eps)
    a = a0
    for _ in range(3):
        t0 = oc.age(a, H0, Om, OL)
        ah = oc.scale_factor(t0 + 0.5 * f * t0, H0, Om, OL)
        a1 = oc.scale_factor(t0 + f * t0, H0, Om, OL)
        k1 = oc.kick_drift(a, ah, H0, Om, OL)[0]
        k2 = oc.kick_drift(ah, a1, H0, Om, OL)[0]
        d = oc.kick_drift(a, a1, H0, Om, OL)[1]
        po = integrate.kick(po, Fo, k1)
        xo = integrate.drift(xo, po, m, d, 1.0)
        Fo = o_p3m.p3m_force(xo, m, 1.0, grid, 1.25, 4.5, eps)
        po = integrate.kick(po, Fo, k2)
        a = a1
    dx = np.abs(xg - xo)
    dx = np.minimum(dx, 1.0 - dx)
    assert np.max(dx) <= 1e-10 / grid
    assert np.max(np.abs(pg - po)) <= 1e-9 * np.max(np.abs(po))
    assert np.max(np.abs(po)) > 0


# --------------------------------------------------------------- pair counts

@pytest.mark.parametrize("name,grid,n", [("uniform", 32, 32768), ("uniform", 16, 1000),
                                         ("uniform", 64, 777)])
def test_pair_count_exact(name, grid, n):
    pos = ics.uniform(n, seed=grid + n)
    rs, rc = o_p3m.params_from_cells(1.0, grid, 1.25, 4.5)
    ref = o_pp.count_pairs(pos, 1.0, rc)
    with plan(grid, n, "fp64") as P:
        assert P.pair_count(dev(pos)) == ref
    with plan(grid, n, "fp32") as P:
        got = P.pair_count(dev(pos))
    assert abs(got - ref) <= max(2, ref * 1e-6)     # FP32 may flip pairs at r = r_c


# --------------------------------------------------------------- forces, small workload

@pytest.fixture(scope="module")
def uniform32():
    w = ics.workload("uniform32")
    pos = workload_positions("uniform32")
    _, a_pp, a_pm = oracle_parts("uniform32")
    return w, pos, a_pp, a_pm


def _plan_for(w, precision):
    return plan(w.grid_n, w.n, precision, rs_cells=w.rs_cells, cutoff_rs=w.cutoff_rs,
                softening=w.softening, G=w.G, box=w.box)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_pp_force_parity(uniform32, precision, tol):
    w, pos, a_pp, _ = uniform32
    with _plan_for(w, precision) as P:
        F = host(P.pp_force(dev(pos), w.mass))
    e = _err(F, a_pp * w.mass)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("soft_cells", [0.0, 0.03, 0.3, 1.0])
def test_pp_force_parity_across_softening(precision, tol, soft_cells):
    """The short-range sum for no softening, the default (0.03 mean spacing)
    and softenings wide against a split-table bin, where the FP32 table is
    taken over r instead of the softened distance; close pairs (0.05-0.2
    cells apart) included."""
    from paper_1510_07621_amd import binding
    grid = 16
    h = 1.0 / grid
    rng = np.random.default_rng(31)
    base = ics.uniform(3500, seed=32)
    near = (base[:, :300] + rng.uniform(0.05, 0.2, (3, 300)) * h) % 1.0
    pos = np.concatenate([base, near], axis=1)
    eps = soft_cells * h
    _, (var, _, _) = binding.split_table(4.5, eps / (1.25 * h))
    assert var == (1 if soft_cells <= 0.03 else 0)
    m = 1.0 / pos.shape[1]
    ref = o_pp.pp_accel(pos, m, 1.0, 1.25 * h, 4.5 * 1.25 * h, eps, 1.0) * m
    with plan(grid, pos.shape[1], precision, softening=eps) as P:
        F = host(P.pp_force(dev(pos), m))
    e = _err(F, ref)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_pm_force_parity(uniform32, precision, tol):
    w, pos, _, a_pm = uniform32
    with _plan_for(w, precision) as P:
        F = host(P.pm_force(dev(pos), w.mass))
    e = _err(F, a_pm * w.mass)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
@pytest.mark.parametrize("fd_order,deconv_power", [(2, 2), (4, 0), (2, 0)])
def test_pm_force_parity_gradient_order_and_deconvolution(precision, tol, fd_order,
                                                          deconv_power):
    """The plan's other mesh options, the 2-point gradient and the Green's
    function without the CIC deconvolution, against the oracle's, in a box
    of side 1.5 on a 32^3 grid with per-particle masses."""
    grid, box, n = 32, 1.5, 6000
    rng = np.random.default_rng(71)
    pos = ics.uniform(n, box, seed=72)
    m = rng.uniform(0.5, 1.5, n) / n
    r_s = 1.25 * box / grid
    ref = o_pm.pm_accel(pos, m, box, grid, r_s, 1.0, fd_order=fd_order,
                        deconv_power=deconv_power) * m
    with plan(grid, n, precision, box=box, fd_order=fd_order,
              deconv_power=deconv_power) as P:
        F = host(P.pm_force(dev(pos), dev(m)))
    e = _err(F, ref)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision,tol,tight", [("fp64", 1e-6, 1e-10), ("fp32", 1e-3, 1e-4)])
def test_p3m_force_parity(uniform32, precision, tol, tight):
    w, pos, a_pp, a_pm = uniform32
    ref = (a_pp + a_pm) * w.mass
    with _plan_for(w, precision) as P:
        F64 = host(P.force(dev(pos), w.mass))
        F32 = host(P.force(dev(pos), w.mass, fp32_out=True))
    e = _err(F64, ref)
    assert e["rms"] <= tol and e["rms"] <= tight, e
    assert e["max"] <= 100 * tight, e
    assert _err(F32, ref)["rms"] <= max(tol, 1e-6)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_plan_sized_for_more_particles_than_the_call(uniform32, precision, tol):
    """The i-group edge is chosen from the plan's n_max (for a mean of 64
    particles per group at n_max): a plan made for 16x the particles, and so
    with smaller groups than the call's density would get, still gives the
    oracle's force (the groups change only the work split), and so does a
    plan for a single particle more than the call (larger groups)."""
    w, pos, a_pp, a_pm = uniform32
    ref = (a_pp + a_pm) * w.mass
    for n_max in (16 * w.n, w.n + 1):
        with plan(w.grid_n, n_max, precision, box=w.box, rs_cells=w.rs_cells,
                  cutoff_rs=w.cutoff_rs, softening=w.softening, G=w.G) as P:
            F = host(P.force(dev(pos), w.mass))
        e = _err(F, ref)
        assert e["rms"] <= tol, (n_max, e)


def test_p3m_method_error_matches_the_oracle_against_ewald(uniform32):
    """P3M vs direct Ewald: the GPU's method error equals the oracle's to
    three significant digits (it is the same discretisation)."""
    w, pos, a_pp, a_pm = uniform32
    tg = sample_targets(pos, 256, seed=5)
    truth = ewald.ewald_accel(pos, w.mass, w.box, eps=w.softening, targets=tg)
    oracle_err = _err((a_pp + a_pm)[:, tg], truth)["rms"]
    with _plan_for(w, "fp64") as P:
        F = host(P.force(dev(pos), w.mass))
    gpu_err = _err(F[:, tg] / w.mass, truth)["rms"]
    assert 1e-3 < oracle_err < 3e-2
    assert abs(gpu_err - oracle_err) <= 5e-4 * oracle_err


# --------------------------------------------------------------- edge cases

def test_empty_and_single_particle():
    with plan(16, 4, "fp64") as P:
        empty = torch.empty((3, 0), dtype=torch.float64, device="cuda")
        out = P.force(empty, 1.0)
        assert out.shape == (3, 0)
        one = dev(np.array([[0.3], [0.7], [0.11]]))
        assert np.max(np.abs(host(P.force(one, 2.0)))) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("box", [1.0, 2.7])
@pytest.mark.parametrize("soft_cells", [0.0, 0.03, 0.3])
def test_lone_particle_short_range_force_is_exactly_zero(precision, box, soft_cells):
    """A particle alone in the box meets only itself: the pair loop must see
    a separation of exactly zero between it and its own staged copy (the
    i-side and j-side relative coordinates formed identically), for cell
    sizes that are and are not powers of two and for both table variables;
    any rounding gap would give it a self-force through the softened weight."""
    grid = 16
    h = box / grid
    for where in ([0.3, 0.7, 0.11], [0.0, 0.5, 0.99999], [0.51, 0.02, 0.73]):
        one = dev(np.array(where)[:, None] * box)
        with plan(grid, 4, precision, box=box, softening=soft_cells * h) as P:
            F = host(P.pp_force(one, 1.7))
        assert np.array_equal(F, np.zeros((3, 1))), (where, F)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_pp_force_parity_box_not_a_power_of_two(precision, tol):
    """The short-range sum in a box of side 2.7 (cell size not a power of
    two), default softening, with close pairs, against the oracle."""
    grid, box = 16, 2.7
    h = box / grid
    rng = np.random.default_rng(41)
    base = ics.uniform(3500, box, seed=42)
    near = (base[:, :300] + rng.uniform(0.05, 0.2, (3, 300)) * h) % box
    pos = np.concatenate([base, near], axis=1)
    eps = 0.03 * h
    m = 1.0 / pos.shape[1]
    ref = o_pp.pp_accel(pos, m, box, 1.25 * h, 4.5 * 1.25 * h, eps, 1.0) * m
    with plan(grid, pos.shape[1], precision, box=box, softening=eps) as P:
        F = host(P.pp_force(dev(pos), m))
    e = _err(F, ref)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dense_cell_ragged_and_masses(precision):
    """300 particles in one cell (several 64-particle chunks), plus a ragged
    uniform background; per-particle masses; compared with the oracle."""
    rng = np.random.default_rng(7)
    grid = 16
    h = 1.0 / grid
    dense = (np.array([5, 9, 15])[:, None] + rng.random((3, 300))) * h   # touches the z face
    pos = np.concatenate([dense, ics.uniform(701, seed=8)], axis=1)
    m = rng.uniform(0.5, 1.5, pos.shape[1]) / pos.shape[1]
    eps = 0.01 * h
    ref = o_p3m.p3m_force(pos, m, 1.0, grid, 1.25, 4.5, eps)
    with plan(grid, pos.shape[1] + 10, precision, softening=eps) as P:
        F = host(P.force(dev(pos), dev(m)))
        Fs = host(P.force(dev(pos), 1.0 / pos.shape[1]))
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert _err(F, ref)["rms"] <= tol
    ref_s = o_p3m.p3m_force(pos, 1.0 / pos.shape[1], 1.0, grid, 1.25, 4.5, eps)
    assert _err(Fs, ref_s)["rms"] <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_heavy_masses_without_softening_and_duplicates(precision, tol):
    """Per-particle masses of order 1e10 (physical units), no softening, and
    exact duplicates: every particle meets its own staged copy and the
    duplicates meet each other at zero separation, where the finite weight of
    the pair loop times a zero separation must stay zero (no overflow of the
    weight times a mass to inf, no inf * 0)."""
    grid = 16
    rng = np.random.default_rng(17)
    base = ics.uniform(1500, seed=18)
    pos = np.concatenate([base, base[:, :40], base[:, 100:103]], axis=1)
    n = pos.shape[1]
    m = rng.uniform(0.5e10, 2e10, n)
    h = 1.0 / grid
    ref = o_pp.pp_accel(pos, m, 1.0, 1.25 * h, 4.5 * 1.25 * h, 0.0, 1.0) * m
    with plan(grid, n, precision, softening=0.0) as P:
        F = host(P.pp_force(dev(pos), dev(m)))
        Fp = host(P.force(dev(pos), dev(m)))
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(Fp))
    e = _err(F, ref)
    assert e["rms"] <= tol, e


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("pair_partials", [0, 80, 1])
def test_one_sided_two_sided_and_overflow_fallback(precision, tol, pair_partials):
    """The short-range sum evaluated from both sides (pair_partials 0), once
    per pair between dense groups with the reactions gathered from partials
    (80 per particle), and with a capacity too small for the input (the
    65536 spare partials only, at 1 per particle, and 4000 more particles
    in one cell: the call falls back to both sides on the device) all match
    the oracle: dense cells of 300, 700 and 500 (groups of several chunks,
    one straddling the z face, two neighbouring), a ragged uniform
    background, per-particle masses and the scalar mass, in a box whose
    cell size is not a power of two."""
    rng = np.random.default_rng(23)
    grid, box = 16, 2.7
    h = box / grid
    cells = [([5, 9, 15], 300), ([5, 9, 0], 700), ([6, 10, 13], 500)]
    if pair_partials == 1:
        cells.append(([11, 2, 7], 4000))
    dense = np.concatenate([(np.array(c)[:, None] + rng.random((3, k))) * h for c, k in cells],
                           axis=1)
    pos = np.concatenate([dense, ics.uniform(1701, box, seed=24)], axis=1)
    n = pos.shape[1]
    m = rng.uniform(0.5, 1.5, n) / n
    eps = 0.02 * h
    r_s = 1.25 * h
    ref = o_pp.pp_accel(pos, m, box, r_s, 4.5 * r_s, eps, 1.0) * m
    ref_s = o_pp.pp_accel(pos, 1.0 / n, box, r_s, 4.5 * r_s, eps, 1.0) / n
    with plan(grid, n, precision, box=box, softening=eps, pair_partials=pair_partials) as P:
        F = host(P.pp_force(dev(pos), dev(m)))
        Fs = host(P.pp_force(dev(pos), 1.0 / n))
        Fp = host(P.force(dev(pos), dev(m)))
        Fpm = host(P.pm_force(dev(pos), dev(m)))
    e = _err(F, ref)
    assert e["rms"] <= tol and e["max"] <= 100 * tol, e
    e = _err(Fs, ref_s)
    assert e["rms"] <= tol and e["max"] <= 100 * tol, e
    assert _err(Fp - Fpm, ref)["rms"] <= 10 * tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_positions_on_faces_and_nodes(precision):
    grid = 32
    h = 1.0 / grid
    pts = np.array([[0.0, 0.0, 0.0], [1.0 - 1e-15, 0.5, 0.25], [3 * h, 7 * h, 31 * h],
                    [0.5, 1.0 - 1e-12, 0.0], [0.999999, 0.999999, 0.999999]]).T
    pos = np.concatenate([pts, ics.uniform(2000, seed=9)], axis=1)
    m = 1.0 / pos.shape[1]
    ref = o_p3m.p3m_force(pos, m, 1.0, grid, 1.25, 4.5, 1e-3)
    with plan(grid, pos.shape[1], precision, softening=1e-3) as P:
        F = host(P.force(dev(pos), m))
    assert _err(F, ref)["rms"] <= (1e-10 if precision == "fp64" else 1e-4)


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lattice_zero_force_and_momentum(precision):
    lat = ics.lattice(32)
    n = lat.shape[1]
    rnd = ics.uniform(n, seed=4)
    with plan(32, n, precision, softening=1e-3) as P:
        F = host(P.force(dev(lat), 1.0 / n))
        Fr = host(P.force(dev(rnd), 1.0 / n))
    scale = np.sqrt(np.mean(np.sum(Fr ** 2, axis=0)))      # typical force of a random set
    assert np.max(np.abs(F)) < (1e-12 if precision == "fp64" else 1e-5) * scale
    tot = np.abs(Fr.sum(axis=1)).max()                     # Newton's third law
    assert tot < (1e-11 if precision == "fp64" else 1e-4) * np.abs(Fr).sum(axis=1).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plane_symmetry_kick_test_of_the_guide(precision):
    """Density varying only along x: no force along y or z."""
    planes = ics.lattice(16)
    planes[0] = (planes[0] + 0.02 * np.sin(2 * np.pi * planes[0])) % 1.0
    with plan(16, planes.shape[1], precision, softening=1e-3) as P:
        F = host(P.force(dev(planes), 1.0 / planes.shape[1]))
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert np.max(np.abs(F[1:])) <= tol * np.max(np.abs(F[0]))


def test_permutation_invariance():
    """The process-count invariance tests of the guide, on one GPU: the same
    particles in another order get the same forces (to rounding)."""
    pos = ics.uniform(8000, seed=12)
    perm = np.random.default_rng(1).permutation(8000)
    with plan(32, 8000, "fp64", softening=1e-3) as P:
        F = host(P.force(dev(pos), 1.0 / 8000))
        Fp = host(P.force(dev(pos[:, perm]), 1.0 / 8000))
    assert _err(Fp, F[:, perm])["rms"] < 1e-12


def test_back_to_back_calls_without_sync_match_separate_calls():
    """The force call forks its mesh part onto the plan's second stream and
    joins it before its last kernel: calls queued back to back (no host
    synchronisation in between, stage timers on) give the forces of calls
    made one at a time, and the mesh-only and pair-only calls in between
    still read a consistent workspace."""
    n = 6000
    xs = [ics.uniform(n, seed=40 + k) for k in range(3)]
    with plan(32, n, "fp64", softening=1e-3) as P:
        ref = []
        for x in xs:
            ref.append(host(P.force(dev(x), 1.0 / n)))
        P.set_timing(8)
        outs = [P.force(dev(x), 1.0 / n) for x in xs]
        pm = P.pm_force(dev(xs[0]), 1.0 / n)
        pp = P.pp_force(dev(xs[1]), 1.0 / n)
        again = P.force(dev(xs[2]), 1.0 / n)
        torch.cuda.synchronize()
        ncall, st = P.stage_times()
        pm_ref = host(P.pm_force(dev(xs[0]), 1.0 / n))
        pp_ref = host(P.pp_force(dev(xs[1]), 1.0 / n))
    for got, want in zip(outs + [again], ref + [ref[2]]):
        assert _err(host(got), want)["max"] < 1e-12
    assert _err(host(pm), pm_ref)["max"] < 1e-12
    assert _err(host(pp), pp_ref)["max"] < 1e-12
    # every stage ran but the gather of reactions (a plan without partials)
    assert ncall == 6 and st["react"] == 0
    assert all(v > 0 for k, v in st.items() if k != "react")


# --------------------------------------------------------------- full-size workloads, sampled

@pytest.mark.parametrize("name,precision,tol,partials,cell_order", [
    ("zeldovich128", "fp32", 1e-3, 0, False), ("zeldovich128", "fp64", 1e-6, 0, False),
    ("plummer256", "fp32", 1e-3, 0, False), ("plummer256", "fp64", 1e-6, 0, False),
    # the benchmark's force call: one-sided sum, force in cell order
    ("plummer256", "fp32", 1e-3, 80, True), ("plummer256", "fp64", 1e-6, 80, False)])
def test_full_size_sampled_parity(name, precision, tol, partials, cell_order):
    w = ics.workload(name)
    pos = workload_positions(name)
    tg, a_pp, a_pm = oracle_parts(name, n_targets=768, seed=3)
    ref = (a_pp + a_pm) * w.mass
    with plan(w.grid_n, w.n, precision, rs_cells=w.rs_cells, cutoff_rs=w.cutoff_rs,
              softening=w.softening, G=w.G, box=w.box, pair_partials=partials) as P:
        if cell_order:
            Fc, order = P.force_cell_order(dev(pos), w.mass)
            order = order.cpu().numpy()
            assert np.array_equal(np.sort(order), np.arange(w.n))
            F = np.empty((3, w.n))
            F[:, order] = host(Fc)
        else:
            F = host(P.force(dev(pos), w.mass))
    e = _err(F[:, tg], ref)
    print(name, precision, e)
    assert e["rms"] <= tol, e
    # per-particle worst case as well (measured: FP32 ~2e-4, FP64 ~2e-13)
    assert e["max"] <= (1e-2 if precision == "fp32" else 1e-9), e
    if precision == "fp64":
        assert e["rms"] <= 1e-10, e
