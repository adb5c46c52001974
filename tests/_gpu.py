"""Shared helpers for the GPU tests: device tensors, plans, and a cache of
oracle results so several tests can compare against one CPU evaluation."""
import functools

import numpy as np
import pytest
import torch

from oracle import p3m as o_p3m
from oracle import pm as o_pm
from oracle import pp as o_pp
from paper_1510_07621_amd import ics


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def plan(grid_n, n_max, precision="fp64", **kw):
    from paper_1510_07621_amd import binding
    return binding.Plan(binding.Params(grid_n=grid_n, precision=precision, **kw), n_max)


@functools.lru_cache(maxsize=8)
def workload_positions(name):
    return ics.workload(name).positions()


@functools.lru_cache(maxsize=32)
def oracle_parts(name, n_targets=None, seed=0):
    """(a_PP, a_PM) of the named workload at a target subset (or all)."""
    w = ics.workload(name)
    pos = workload_positions(name)
    targets = None
    if n_targets is not None:
        targets = sample_targets(pos, n_targets, seed)
    a_pp = o_pp.pp_accel(pos, w.mass, w.box, w.r_s, w.r_c, w.softening, w.G,
                         targets=targets)
    a_pm = o_pm.pm_accel(pos, w.mass, w.box, w.grid_n, w.r_s, w.G, targets=targets)
    return targets, a_pp, a_pm


def sample_targets(pos, k, seed=0):
    rng = np.random.default_rng(1000 + seed)
    n = pos.shape[1]
    return np.sort(rng.choice(n, size=min(k, n), replace=False))


def p3m_ref(pos, mass, grid_n, **kw):
    return o_p3m.p3m_force(pos, mass, 1.0, grid_n, **kw)
