"""The allocation-free short-range force (pp_force_noalloc, no plan, fixed
device workspace) against the plan-based pp_force through the C ABI: two
calls in a row on one GPU, the second with fewer particles (the workspace
keeps the first call's contents), both precisions, a scalar and a
per-particle mass; and its size limits."""
import numpy as np
import pytest
import torch

from oracle import metrics
from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_noalloc_matches_plan_pp_force_on_two_calls(precision, tol):
    from paper_1510_07621_amd import binding
    rng = np.random.default_rng(61)
    grid, eps = 32, 0.03 / 32
    sizes = (20000, 3001)
    for n, use_mass in zip(sizes, (False, True)):
        pos = ics.uniform(n, seed=n)
        dense = (np.array([3, 30, 17])[:, None] + rng.random((3, 150))) / grid
        pos = np.concatenate([pos, dense], axis=1)
        n = pos.shape[1]
        m = dev(rng.uniform(0.5, 1.5, n) / n) if use_mass else 1.0 / n
        prm = binding.Params(grid_n=grid, softening=eps, precision=precision)
        x = dev(pos)
        got = host(binding.pp_force_noalloc(prm, x, m))
        with plan(grid, n, precision, softening=eps) as P:
            want = host(P.pp_force(x, m))
        e = metrics.force_errors(got, want)
        print(precision, n, e)
        assert e["rms"] <= tol and e["max"] <= 100 * tol, e


def test_noalloc_limits_and_errors():
    from paper_1510_07621_amd import binding
    x = dev(ics.uniform(100, seed=1))
    with pytest.raises(ValueError, match="fixed workspace"):
        binding.pp_force_noalloc(binding.Params(grid_n=128), x, 0.01)
    big = torch.zeros((3, 65537), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="fixed workspace"):
        binding.pp_force_noalloc(binding.Params(grid_n=32), big, 1.0)
    with pytest.raises(ValueError):
        binding.pp_force_noalloc(binding.Params(grid_n=24), x, 0.01)       # not a power of two
    empty = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    assert binding.pp_force_noalloc(binding.Params(grid_n=16), empty, 1.0).shape == (3, 0)
