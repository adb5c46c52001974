"""Particles kept in cell order: p3m_force_cell_order and p3m_kick_reorder.

The force of a call in the cell order of its binning is the P3M force of
the same particles (guide Ch. 1), stored at each particle's sorted slot; the
kick that reorders is the oracle's kick (one IEEE double sum per component)
followed by a permutation, so its momenta are compared bit for bit. A
leapfrog run that keeps its particles in cell order between steps, mapped
back to the particles' ids, follows the oracle's run to the force parity.
"""
import numpy as np
import pytest
import torch

from oracle import integrate, metrics
from oracle import p3m as o_p3m
from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _cells(pos, grid):
    c = np.clip(np.floor(pos * grid).astype(np.int64), 0, grid - 1)
    return (c[0] * grid + c[1]) * grid + c[2]


@pytest.mark.parametrize("precision,partials", [("fp64", 0), ("fp64", 80), ("fp32", 0),
                                                ("fp32", 80)])
def test_force_in_cell_order_is_the_force_at_the_sorted_slots(precision, partials):
    """Clustered input (a Plummer mix, so that dense groups take the one-sided
    sum): the order is a permutation that sorts the cells, and the force at
    slot s is the force on particle order[s] (to rounding: the order inside a
    cell may differ between the two calls)."""
    from paper_1510_07621_amd import binding
    grid, n = 32, 40000
    pos = ics.plummer_mix(n, n_spheres=20, frac=0.7, seed=5)
    m = 1.0 / n
    x = dev(pos)
    with plan(grid, n, precision, pair_partials=partials) as P:
        F = host(P.force(x, m))
        Fc, order = P.force_cell_order(x, m)
        Fc, order = host(Fc), order.cpu().numpy()
        with pytest.raises(ValueError):
            P.force_cell_order(x, m, order=torch.empty(n, dtype=torch.int64, device=x.device))
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.all(np.diff(_cells(pos[:, order], grid)) >= 0)
    e = metrics.force_errors(Fc, F[:, order])
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert e["rms"] < tol and e["max"] < 100 * tol, e
    # FP32 force output through the same path
    with plan(grid, n, precision, pair_partials=partials) as P:
        F32, order32 = P.force_cell_order(x, m, fp32_out=True)
        F32, order32 = host(F32).astype(np.float64), order32.cpu().numpy()
    assert np.array_equal(np.sort(order32), np.arange(n))
    e32 = metrics.force_errors(F32, F[:, order32])
    assert e32["rms"] < max(tol, 1e-6), e32


@pytest.mark.parametrize("with_arrays", [False, True])
def test_kick_reorder_bitwise(with_arrays):
    """Momenta: the oracle's kick of the permuted momenta, bit for bit, for
    both force precisions; positions, ids and masses: the permutation."""
    from paper_1510_07621_amd import binding
    n = 70001                                   # not a multiple of the block
    rng = np.random.default_rng(21)
    x = rng.uniform(size=(3, n))
    p = rng.normal(size=(3, n))
    order = rng.permutation(n).astype(np.int32)
    ids = rng.integers(0, 1 << 40, n).astype(np.int64)
    mass = rng.uniform(0.5, 2.0, n)
    for fdt, tdt in ((np.float64, torch.float64), (np.float32, torch.float32)):
        F = rng.normal(size=(3, n)).astype(fdt)
        po, mo, io, ma = binding.kick_reorder(
            torch.as_tensor(order, device="cuda"), dev(x), dev(p), dev(F, tdt), 0.37,
            ids=torch.as_tensor(ids, device="cuda") if with_arrays else None,
            mass=dev(mass) if with_arrays else None)
        assert np.array_equal(host(mo), integrate.kick(p[:, order], F, 0.37))
        assert np.array_equal(host(po), x[:, order])
        if with_arrays:
            assert np.array_equal(io.cpu().numpy(), ids[order])
            assert np.array_equal(host(ma), mass[order])
        else:
            assert io is None and ma is None


def test_kick_reorder_rejects_overlap_and_half_given_arrays():
    from paper_1510_07621_amd import binding
    n = 100
    x = dev(np.random.default_rng(0).uniform(size=(3, n)))
    p = torch.zeros_like(x)
    F = torch.zeros_like(x)
    order = torch.arange(n, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):            # output over an input
        binding.kick_reorder(order, x, p, F, 0.1, out=(x, None, None, None))
    ids = torch.arange(n, dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):            # ids given, ids_out aliased to ids
        binding.kick_reorder(order, x, p, F, 0.1, ids=ids, out=(None, None, ids, None))


@pytest.mark.parametrize("precision,partials", [("fp64", 0), ("fp64", 80)])
def test_leapfrog_in_cell_order_follows_the_oracle(precision, partials):
    """Four kick-drift-kick steps with the particles reordered into cell order
    at every force call, mapped back by id at the end: the oracle's run
    (its own force, kick and drift in input order) to the force parity."""
    from paper_1510_07621_amd import binding
    grid, n, dt = 16, 3000, 1e-4
    pos = ics.plummer_mix(n, n_spheres=6, frac=0.6, seed=3)
    m = 1.0 / n
    eps = 0.03 / grid
    x = dev(pos)
    p = torch.zeros_like(x)
    ids = torch.arange(n, dtype=torch.int64, device="cuda")
    with plan(grid, n, precision, softening=eps, pair_partials=partials) as P:
        F, order = P.force_cell_order(x, m)
        x, p, ids, _ = binding.kick_reorder(order, x, p, F, 0.0, ids=ids)
        for _ in range(4):
            binding.kick_drift(x, p, F, m, 0.5 * dt, dt, 1.0)
            P.force_cell_order(x, m, out=F, order=order)
            x, p, ids, _ = binding.kick_reorder(order, x, p, F, 0.5 * dt, ids=ids)
        idh = ids.cpu().numpy()
        xg = np.empty((3, n)); pg = np.empty((3, n))
        xg[:, idh] = host(x)
        pg[:, idh] = host(p)
    assert np.array_equal(np.sort(idh), np.arange(n))
    xo, po = pos.copy(), np.zeros_like(pos)
    Fo = o_p3m.p3m_force(xo, m, 1.0, grid, 1.25, 4.5, eps)
    for _ in range(4):
        po = integrate.kick(po, Fo, 0.5 * dt)
        xo = integrate.drift(xo, po, m, dt, 1.0)
        Fo = o_p3m.p3m_force(xo, m, 1.0, grid, 1.25, 4.5, eps)
        po = integrate.kick(po, Fo, 0.5 * dt)
    dx = np.abs(xg - xo)
    dx = np.minimum(dx, 1.0 - dx)
    assert np.max(dx) <= 1e-10 / grid
    assert np.max(np.abs(pg - po)) <= 1e-9 * np.max(np.abs(po))


@pytest.mark.parametrize("n", [1, 2, 63, 65])
def test_cell_order_small_and_ragged_sets(n):
    """A handful of particles (one, two, a wave's worth minus and plus one):
    the order is a permutation sorting the cells, the force at each slot is
    p3m_force's for that particle, and the reordering kick of that force is
    the oracle's kick, bit for bit."""
    from paper_1510_07621_amd import binding
    grid = 16
    pos = ics.uniform(n, seed=40 + n)
    m = 1.0 / max(n, 1)
    x = dev(pos)
    with plan(grid, max(n, 1), "fp64", pair_partials=80) as P:
        F = host(P.force(x, m))
        Fc, order = P.force_cell_order(x, m)
        Fc, order = host(Fc), order.cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.all(np.diff(_cells(pos[:, order], grid)) >= 0)
    assert np.allclose(Fc, F[:, order], rtol=1e-12, atol=1e-12 * np.abs(F).max())
    p = np.random.default_rng(n).normal(size=(3, n))
    po, mo, _, _ = binding.kick_reorder(torch.as_tensor(order, device="cuda"), x, dev(p),
                                        dev(Fc), 0.25)
    assert np.array_equal(host(mo), integrate.kick(p[:, order], Fc, 0.25))
    assert np.array_equal(host(po), pos[:, order])
