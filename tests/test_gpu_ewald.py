"""GPU PP-with-Ewald (pp_ewald_force, p3m_ewald_correction) against O-EW.

The plan tabulates the Ewald correction c(r) = e(r) - r/|r|^3 on the
ewald_gridsize^3 node grid; O-EW gives e(r) directly (a unit source at the
origin seen from r, no table). At table nodes the interpolation is exact, so
the table entries and any force whose pair separations are all node vectors
agree with O-EW to rounding; between nodes the trilinear interpolation error
is measured (it falls as the square of the node spacing).
"""
import numpy as np
import pytest

from oracle import ewald, metrics
from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _c_ref(r, box):
    """c(r) from O-EW: a massless test particle at r, unit mass at the origin."""
    n = r.shape[1]
    pos = np.concatenate([np.zeros((3, 1)), np.mod(r, box)], axis=1)
    m = np.concatenate([[1.0], np.zeros(n)])
    a = ewald.ewald_accel(pos, m, box, G=1.0, targets=np.arange(1, n + 1))
    d = r - box * np.round(r / box)
    newton = d / np.linalg.norm(d, axis=0) ** 3
    return -a - newton


@pytest.mark.parametrize("E", [16, 64])
def test_table_nodes_match_direct_ewald(E):
    box = 2.0
    rng = np.random.default_rng(81)
    nodes = rng.integers(-E // 2, E // 2, (3, 300))
    nodes = nodes[:, np.any(nodes != 0, axis=0)]
    r = nodes * (box / E)
    ref = _c_ref(r, box)
    with plan(16, 8, "fp64", box=box, ewald_gridsize=E) as P:
        got = host(P.ewald_correction(dev(r)))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale


def test_table_interpolation_error_falls_with_the_spacing():
    box = 1.0
    r = (np.random.default_rng(82).random((3, 400)) - 0.5) * box
    ref = _c_ref(r, box)
    errs = []
    for E in (16, 32, 64):
        with plan(16, 8, "fp64", ewald_gridsize=E) as P:
            got = host(P.ewald_correction(dev(r)))
        errs.append(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert errs[2] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0     # second order


def test_pp_ewald_force_on_node_separations_is_exact():
    """Particles on random sites of the table's node lattice (so every pair
    separation is a node vector), random masses, softening 0: the table
    interpolation is exact and the force equals O-EW to rounding."""
    E, box = 32, 1.0
    rng = np.random.default_rng(83)
    sites = rng.choice(E ** 3, size=1500, replace=False)
    pos = np.stack(np.unravel_index(sites, (E, E, E))).astype(np.float64) * (box / E)
    m = rng.uniform(0.5, 1.5, pos.shape[1]) / pos.shape[1]
    ref = ewald.ewald_force(pos, m, box, G=1.0)
    with plan(16, pos.shape[1], "fp64", ewald_gridsize=E) as P:
        F = host(P.pp_ewald_force(dev(pos), dev(m)))
    assert metrics.force_errors(F, ref)["rms"] <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 63, 65, 600])
def test_pp_ewald_force_ragged_sizes(n):
    """Sizes below one block of 64 i-particles, one past it, and a j tile of
    600 entries (9 * 64 + 24), where six of the sixteen waves of a block have
    no entries: node-lattice sites as above, so the force equals O-EW to
    rounding. A lone particle feels nothing: its periodic images and the
    neutralising background balance by symmetry, and it has no pairs."""
    E, box = 32, 1.0
    rng = np.random.default_rng(86 + n)
    sites = rng.choice(E ** 3, size=n, replace=False)
    pos = np.stack(np.unravel_index(sites, (E, E, E))).astype(np.float64) * (box / E)
    m = rng.uniform(0.5, 1.5, n) / n
    with plan(16, n, "fp64", ewald_gridsize=E) as P:
        F = host(P.pp_ewald_force(dev(pos), dev(m)))
    if n == 1:
        assert np.all(F == 0.0)
        return
    ref = ewald.ewald_force(pos, m, box, G=1.0)
    assert metrics.force_errors(F, ref)["rms"] <= 1e-10


def test_pp_ewald_force_uniform32():
    """The 32^3 uniform workload with its softening (0.03 mean spacing):
    pp_ewald_force with a 64^3 table against O-EW on 256 sampled particles."""
    w = ics.workload("uniform32")
    pos = w.positions()
    tg = np.sort(np.random.default_rng(84).choice(w.n, 256, replace=False))
    ref = ewald.ewald_force(pos, w.mass, w.box, G=1.0, eps=w.softening, targets=tg)
    with plan(w.grid_n, w.n, "fp64", softening=w.softening, ewald_gridsize=64) as P:
        F = host(P.pp_ewald_force(dev(pos), w.mass))
        F32 = host(P.pp_ewald_force(dev(pos), w.mass, fp32_out=True))
    e = metrics.force_errors(F[:, tg], ref)
    assert e["rms"] <= 1e-4, e
    assert metrics.force_errors(F32[:, tg], F[:, tg])["rms"] <= 1e-6


def test_pp_ewald_argument_errors():
    pos = dev(ics.uniform(10, seed=85))
    with plan(16, 10, "fp64") as P:                   # no table
        with pytest.raises(ValueError):
            P.pp_ewald_force(pos, 0.1)
        with pytest.raises(ValueError):
            P.ewald_correction(pos)
    from paper_1510_07621_amd import binding
    for E in (6, 7, 1024):
        with pytest.raises(ValueError):
            binding.Plan(binding.Params(grid_n=16, ewald_gridsize=E), 10)
